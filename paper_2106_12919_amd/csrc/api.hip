// C ABI of libpic (include/pic.h): context, validation, table upload and the
// orchestration of one hybrid PSATD PIC cycle (Sec. 2) from the HIP kernels.
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/pic.h"
#include "kernels.h"

using namespace pic;

// Scratch of pic_deposit_noalloc: the per-call tile sort of each species (the slot of every
// particle and its inverse, two int32 per particle) for callers that cannot allocate device
// memory.  A file-scope device array: each GPU the library runs on holds its own copy until the
// process ends, and every call on that GPU shares it.  Host code reaches it only through the
// per-device address hipGetSymbolAddress returns (scratch_address below), never by its name.
constexpr size_t kNoAllocScratchBytes = size_t(32) << 20;
constexpr int64_t kNoAllocMaxParticles = (int64_t)(kNoAllocScratchBytes / (2 * sizeof(int)));
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

thread_local std::string g_init_error;

// Device address of `scratch` on each device, taken once per device with that device current.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

void* scratch_address(int dev, std::string& err) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (dev < 0 || dev >= kMaxDevices) {
    err = "device index beyond the scratch table";
    return nullptr;
  }
  if (!g_scratch_ptr[dev]) {
    void* q = nullptr;
    const hipError_t e = hipGetSymbolAddress(&q, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !q) {
      (void)hipGetLastError();
      err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
      return nullptr;
    }
    g_scratch_ptr[dev] = q;
  }
  return g_scratch_ptr[dev];
}

const char* const kStageNames[] = {"center_s2n",   "gather_push", "deposit",       "center_n2s", "fft_forward",
                                   "psatd_update", "fft_inverse", "entry_forward", "tile_sort",  "clear_sources",
                                   "deposit_reduce", "exit_inverse"};
constexpr int kNumStages = 12;
enum Stage {
  ST_S2N = 0, ST_PUSH, ST_DEPOSIT, ST_N2S, ST_FFT_FWD, ST_UPDATE, ST_FFT_INV, ST_ENTRY, ST_SORT, ST_CLEAR, ST_REDUCE,
  ST_EXIT
};

struct EventPair {
  hipEvent_t a, b;
  int stage;
};

struct EngineBase {
  virtual ~EngineBase() = default;
};

bool factor23(int n) {
  if (n <= 0) return false;
  while (n % 2 == 0) n /= 2;
  while (n % 3 == 0) n /= 3;
  return n == 1;
}

}  // namespace

struct pic_ctx_s {
  pic_params p{};
  hipStream_t stream = nullptr;
  int device = 0;
  std::string err;
  std::unique_ptr<EngineBase> eng;
  std::vector<double> ccoef;  // alpha^s_{m,n}/2 for the centering order
  // profiling
  bool profiling = false;
  std::vector<EventPair> pending;
  std::vector<EventPair> pool;
  double stage_ms[kNumStages] = {0};
  int64_t stage_count[kNumStages] = {0};
  double* d_acc = nullptr;  // 2 doubles for reductions
  int* d_bad = nullptr;     // count of particles skipped for an out-of-range cell index
  void* noalloc = nullptr;  // this device's copy of `scratch` (pic_deposit_noalloc), or null
  std::string noalloc_err;

  pic_status fail(pic_status s, const std::string& msg) {
    err = msg;
    return s;
  }
  pic_status check(const char* where) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(PIC_EHIP, std::string(where) + ": " + hipGetErrorString(e));
    return PIC_OK;
  }
  void stage_begin(int st, EventPair& ev) {
    if (!profiling) return;
    if (pool.empty()) {
      EventPair e{};
      (void)hipEventCreate(&e.a);
      (void)hipEventCreate(&e.b);
      pool.push_back(e);
    }
    ev = pool.back();
    pool.pop_back();
    ev.stage = st;
    (void)hipEventRecord(ev.a, stream);
  }
  void stage_end(EventPair& ev) {
    if (!profiling) return;
    (void)hipEventRecord(ev.b, stream);
    pending.push_back(ev);
  }
  void collect() {
    for (auto& ev : pending) {
      float ms = 0;
      if (hipEventSynchronize(ev.b) == hipSuccess && hipEventElapsedTime(&ms, ev.a, ev.b) == hipSuccess) {
        stage_ms[ev.stage] += ms;
        stage_count[ev.stage] += 1;
      }
      pool.push_back(ev);
    }
    pending.clear();
  }
};

namespace {

struct StageScope {
  pic_ctx_s* c;
  EventPair ev{};
  StageScope(pic_ctx_s* c_, int st) : c(c_) { c->stage_begin(st, ev); }
  ~StageScope() { c->stage_end(ev); }
};

// Per-species particle scratch: a second set of SoA arrays (ping-pong with the
// caller's arrays while pic_step keeps particles in tile order) and sort indices.
template <typename T>
struct SpeciesScratch {
  int64_t cap = 0;
  int32_t* cell = nullptr;
  T* off[3] = {nullptr, nullptr, nullptr};
  T* u[3] = {nullptr, nullptr, nullptr};
  T* w = nullptr;
  int* dst = nullptr;
  int* perm = nullptr;
  // tile groupings of pic_step: counts[ntiles + 1], starts[ntiles + 2] (two, alternating)
  int* counts[2] = {nullptr, nullptr};
  int* starts[2] = {nullptr, nullptr};
  int* cursor = nullptr;
  int* nbr = nullptr;       // [27 * ntiles]: per tile, particles per neighbour tile (from the deposition)
  int* nbr_base = nullptr;  // [27 * ntiles]: per tile, first slot of its run in each neighbour tile
};

template <typename T>
struct Engine : EngineBase {
  Fft3D<T> fft;
  PsatdTables<T> tab;
  TileGeom tiles{};
  int* t_counts = nullptr;  // ntiles + 1
  int* t_starts = nullptr;  // ntiles + 2
  int* t_cursor = nullptr;  // ntiles + 1
  int* work = nullptr;      // tile counter of the persistent deposition
  T* stage = nullptr;       // per-tile deposition boxes, ntiles * 4 * deposit_stage_slot
  T* astage = nullptr;      // per-tile boxes of the reverse mode's scatter, ntiles * 6 * deposit_box^3 (on first use)
  // rho, J of particles past their tile's box (zero between depositions), the two flags that
  // say whether a deposition spilled, and the count of depositions that chose between them
  T* spill[4] = {nullptr, nullptr, nullptr, nullptr};
  int* spill_flag = nullptr;
  int* box_faces = nullptr;  // per tile, the outer faces of its deposition box that were staged
  unsigned dep_k = 0;
  std::vector<SpeciesScratch<T>> sps;
  cplx<T>* Eh[3] = {nullptr, nullptr, nullptr};
  cplx<T>* Bh[3] = {nullptr, nullptr, nullptr};
  cplx<T>* Jh[3] = {nullptr, nullptr, nullptr};
  cplx<T>* rh[2] = {nullptr, nullptr};
  cplx<T>* scratch[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  cplx<T>* Ah[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};  // averaged <E>, <B> spectra
  T* tmp = nullptr;
  std::vector<void*> allocs;

  ~Engine() override {
    for (void* a : allocs) (void)hipFree(a);
    fft.release();
  }
  template <typename P>
  hipError_t alloc(P** out, size_t count) {
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, count * sizeof(P) > 0 ? count * sizeof(P) : 1);
    if (e != hipSuccess) return e;
    allocs.push_back(q);
    *out = reinterpret_cast<P*>(q);
    return hipSuccess;
  }
  hipError_t release_one(void* q) {
    for (size_t i = 0; i < allocs.size(); ++i)
      if (allocs[i] == q) {
        allocs.erase(allocs.begin() + i);
        return hipFree(q);
      }
    return hipSuccess;
  }
  // grows the scratch of species s to n particles
  hipError_t ensure_species(size_t s, int64_t n) {
    if (sps.size() <= s) sps.resize(s + 1);
    SpeciesScratch<T>& x = sps[s];
    if (x.cap >= n) return hipSuccess;
    void* old[17] = {x.cell, x.off[0], x.off[1], x.off[2], x.u[0], x.u[1], x.u[2], x.w, x.dst, x.perm,
                     x.counts[0], x.counts[1], x.starts[0], x.starts[1], x.cursor, x.nbr, x.nbr_base};
    for (void* q : old)
      if (q) (void)release_one(q);
    x = SpeciesScratch<T>{};
    hipError_t e;
    const size_t m = (size_t)(n > 0 ? n : 1);
    const size_t nt = (size_t)tiles.ntiles;
    for (int b = 0; b < 2; ++b) {
      if ((e = alloc(&x.counts[b], nt + 1)) != hipSuccess) return e;
      if ((e = alloc(&x.starts[b], nt + 2)) != hipSuccess) return e;
    }
    if ((e = alloc(&x.cursor, nt + 1)) != hipSuccess) return e;
    if ((e = alloc(&x.nbr, 27 * nt)) != hipSuccess) return e;
    if ((e = alloc(&x.nbr_base, 27 * nt)) != hipSuccess) return e;
    if ((e = alloc(&x.cell, m)) != hipSuccess) return e;
    for (int d = 0; d < 3; ++d) {
      if ((e = alloc(&x.off[d], m)) != hipSuccess) return e;
      if ((e = alloc(&x.u[d], m)) != hipSuccess) return e;
    }
    if ((e = alloc(&x.w, m)) != hipSuccess) return e;
    if ((e = alloc(&x.dst, m)) != hipSuccess) return e;
    if ((e = alloc(&x.perm, m)) != hipSuccess) return e;
    x.cap = n;
    return hipSuccess;
  }
  template <typename P>
  hipError_t upload(P** out, const std::vector<P>& h) {
    hipError_t e = alloc(out, h.size());
    if (e != hipSuccess) return e;
    return hipMemcpy(*out, h.data(), h.size() * sizeof(P), hipMemcpyHostToDevice);
  }
};

template <typename T>
hipError_t build_engine(const pic_params& p, Engine<T>& e) {
  hipError_t err = e.fft.init(p.nx, p.ny, p.nz);
  if (err != hipSuccess) return err;
  const int n[3] = {p.nx, p.ny, p.nz};
  const double d[3] = {p.dx, p.dy, p.dz};
  const int nzh = e.fft.nzh;
  const int m = p.center_order / 2;
  std::vector<double> calpha(m);
  alpha_staggered(m, calpha.data());
  for (double& v : calpha) v *= 0.5;
  // per-axis [k]_s and the staggered phase operators D+- = i [k]_s exp(+-i k d / 2)
  // (nodal solver: the centered [k]_c and D+- = i [k]_c, no half-cell phase)
  const bool nodal = (p.flags & PIC_NODAL_SOLVER) != 0;
  std::vector<double> ks[3];
  for (int a = 0; a < 3; ++a) {
    ks[a].resize(n[a]);
    if (nodal)
      k_centered_axis(n[a], d[a], p.psatd_order, ks[a].data());
    else
      k_staggered_axis(n[a], d[a], p.psatd_order, ks[a].data());
    const int len = (a == 2) ? nzh : n[a];
    std::vector<cplx<T>> dp(len), dm(len);
    const double two_pi = 6.283185307179586476925286766559;
    for (int i = 0; i < len; ++i) {
      const int f = (i <= (n[a] - 1) / 2) ? i : i - n[a];
      const double k = two_pi * f / (n[a] * d[a]);
      const double sh = nodal ? 0.0 : std::sin(0.5 * k * d[a]), ch = nodal ? 1.0 : std::cos(0.5 * k * d[a]);
      // Nodal solver, Nyquist index of an even axis: the odd operator i [k]_c has no
      // real-valued action on that self-conjugate mode (finite orders give [k]_c = 0
      // there anyway; at infinite order the derivative is dropped, omega keeps |k|).
      const double kd = (nodal && 2 * i == n[a]) ? 0.0 : ks[a][i];
      dp[i] = cmake((T)(-kd * sh), (T)(kd * ch));
      dm[i] = cmake((T)(kd * sh), (T)(kd * ch));
    }
    if ((err = e.upload(&e.tab.Dp[a], dp)) != hipSuccess) return err;
    if ((err = e.upload(&e.tab.Dm[a], dm)) != hipSuccess) return err;
    // Fourier symbol of the nodes -> centres centering along this axis, in the index-space
    // DFT convention: sum_n c_n (e^{i th n} + e^{-i th (n-1)}), th = 2 pi f / n, c_n = alpha^s_{m,n}/2
    std::vector<cplx<T>> tc(len);
    for (int i = 0; i < len; ++i) {
      const int f = (i <= (n[a] - 1) / 2) ? i : i - n[a];
      const double th = two_pi * f / n[a];
      double re = 0, im = 0;
      for (int q = 1; q <= m; ++q) {
        re += calpha[q - 1] * (std::cos(th * q) + std::cos(th * (q - 1)));
        im += calpha[q - 1] * (std::sin(th * q) - std::sin(th * (q - 1)));
      }
      tc[i] = cmake((T)re, (T)im);
    }
    if ((err = e.upload(&e.tab.Tc[a], tc)) != hipSuccess) return err;
  }
  // 3D per-mode tables on the unpadded half spectrum
  const size_t M = (size_t)p.nx * p.ny * nzh;
  std::vector<T> C(M), Sw(M), X1(M), X2(M), X3(M);
  for (int i = 0; i < p.nx; ++i)
    for (int j = 0; j < p.ny; ++j)
      for (int k = 0; k < nzh; ++k) {
        const size_t idx = ((size_t)i * p.ny + j) * nzh + k;
        const double w = std::sqrt(ks[0][i] * ks[0][i] + ks[1][j] * ks[1][j] + ks[2][k] * ks[2][k]);
        double c, s, x1, x2, x3;
        psatd_coefficients(w, p.dt, &c, &s, &x1, &x2, &x3);
        C[idx] = (T)c;
        Sw[idx] = (T)s;
        X1[idx] = (T)x1;
        X2[idx] = (T)x2;
        X3[idx] = (T)x3;
      }
  if ((err = e.upload(&e.tab.C, C)) != hipSuccess) return err;
  if ((err = e.upload(&e.tab.Sw, Sw)) != hipSuccess) return err;
  if ((err = e.upload(&e.tab.X1, X1)) != hipSuccess) return err;
  if ((err = e.upload(&e.tab.X2, X2)) != hipSuccess) return err;
  if ((err = e.upload(&e.tab.X3, X3)) != hipSuccess) return err;
  e.tab.cc = (p.flags & PIC_CURRENT_CORRECTION) != 0;
  e.tab.inv_dt = (T)(1.0 / p.dt);
  if (p.v_gal[0] != 0 || p.v_gal[1] != 0 || p.v_gal[2] != 0 || (p.flags & PIC_AVERAGED)) {
    // standard Galilean PSATD (Sec. 4.3): W = v_gal . [k]_c per mode; averaged (Sec. 4.4) too
    std::vector<double> kc[3];
    for (int a = 0; a < 3; ++a) {
      kc[a].resize(n[a]);
      k_centered_axis(n[a], d[a], p.psatd_order, kc[a].data());
    }
    const bool avg = (p.flags & PIC_AVERAGED) != 0;
    std::vector<cplx<T>> G[6], Av[6];
    for (auto& v : G) v.resize(M);
    if (avg)
      for (auto& v : Av) v.resize(M);
    // x-planes of modes spread over the host's threads (quadrature per mode)
    auto plane = [&](int i) {
      std::complex<double> g[6];
      for (int j = 0; j < p.ny; ++j)
        for (int k = 0; k < nzh; ++k) {
          const size_t idx = ((size_t)i * p.ny + j) * nzh + k;
          const double w = std::sqrt(ks[0][i] * ks[0][i] + ks[1][j] * ks[1][j] + ks[2][k] * ks[2][k]);
          const double W = p.v_gal[0] * kc[0][i] + p.v_gal[1] * kc[1][j] + p.v_gal[2] * kc[2][k];
          galilean_coefficients(w, W, p.dt, g);
          for (int q = 0; q < 6; ++q) G[q][idx] = cmake((T)g[q].real(), (T)g[q].imag());
          if (avg) {
            averaged_coefficients(w, W, p.dt, g);
            for (int q = 0; q < 6; ++q) Av[q][idx] = cmake((T)g[q].real(), (T)g[q].imag());
          }
        }
    };
    const int nth = std::max(1, std::min(std::min(p.nx, 16), (int)std::thread::hardware_concurrency()));
    std::vector<std::thread> pool;
    for (int t = 0; t < nth; ++t)
      pool.emplace_back([&, t] {
        for (int i = t; i < p.nx; i += nth) plane(i);
      });
    for (auto& th : pool) th.join();
    for (int q = 0; q < 6; ++q)
      if ((err = e.upload(&e.tab.G[q], G[q])) != hipSuccess) return err;
    if (avg)
      for (int q = 0; q < 6; ++q)
        if ((err = e.upload(&e.tab.Av[q], Av[q])) != hipSuccess) return err;
  }
  // spectra and scratch, zeroed once (padding columns stay zero)
  const size_t ns = e.fft.spectrum_elems();
  cplx<T>** bufs[17] = {&e.Eh[0], &e.Eh[1], &e.Eh[2], &e.Bh[0], &e.Bh[1], &e.Bh[2], &e.Jh[0], &e.Jh[1], &e.Jh[2],
                        &e.rh[0], &e.rh[1], &e.scratch[0], &e.scratch[1], &e.scratch[2], &e.scratch[3],
                        &e.scratch[4], &e.scratch[5]};
  for (auto b : bufs) {
    if ((err = e.alloc(b, ns)) != hipSuccess) return err;
    if ((err = hipMemset(*b, 0, ns * sizeof(cplx<T>))) != hipSuccess) return err;
  }
  if (p.flags & PIC_AVERAGED)
    for (int q = 0; q < 6; ++q) {
      if ((err = e.alloc(&e.Ah[q], ns)) != hipSuccess) return err;
      if ((err = hipMemset(e.Ah[q], 0, ns * sizeof(cplx<T>))) != hipSuccess) return err;
    }
  if ((err = e.alloc(&e.tmp, (size_t)p.nx * p.ny * p.nz)) != hipSuccess) return err;
  for (int q = 0; q < 4; ++q) {
    if ((err = e.alloc(&e.spill[q], (size_t)p.nx * p.ny * p.nz)) != hipSuccess) return err;
    if ((err = hipMemset(e.spill[q], 0, (size_t)p.nx * p.ny * p.nz * sizeof(T))) != hipSuccess) return err;
  }
  if ((err = e.alloc(&e.spill_flag, 2)) != hipSuccess) return err;
  if ((err = hipMemset(e.spill_flag, 0, 2 * sizeof(int))) != hipSuccess) return err;
  // deposition tiles of kTile^3 = 8^3 cells: the LDS box of 4 components is at most
  // 4 * 13^3 * 8 B = 70 KiB (FP64, cubic); the gather box 13^3 nodes * 6 components
  const GridGeom g = make_geom(p.nx, p.ny, p.nz, p.dx, p.dy, p.dz, p.dt, p.shape_order);
  e.tiles = make_tiles(g);
  if ((err = e.alloc(&e.tiles.scan_tmp, (size_t)(e.tiles.ntiles + 1) / 8192 + 2)) != hipSuccess) return err;
  if ((err = e.alloc(&e.box_faces, (size_t)e.tiles.ntiles)) != hipSuccess) return err;
  if ((err = e.alloc(&e.t_counts, (size_t)e.tiles.ntiles + 1)) != hipSuccess) return err;
  if ((err = e.alloc(&e.t_starts, (size_t)e.tiles.ntiles + 2)) != hipSuccess) return err;
  if ((err = e.alloc(&e.t_cursor, (size_t)e.tiles.ntiles + 1)) != hipSuccess) return err;
  if ((err = e.alloc(&e.work, 1)) != hipSuccess) return err;
  // the row layout of deposit_tiled (B x B x 16 per component) holds the node-major boxes
  // (B^3) of the staggered cycle's deposition too
  const size_t slot = (size_t)deposit_stage_slot(p.shape_order);
  if ((err = e.alloc(&e.stage, (size_t)e.tiles.ntiles * 4 * slot)) != hipSuccess) return err;
  return hipSuccess;
}

pic_status validate_params(const pic_params* p, std::string& msg) {
  if (!p) { msg = "params is NULL"; return PIC_EINVAL; }
  const int n[3] = {p->nx, p->ny, p->nz};
  for (int a = 0; a < 3; ++a) {
    if (n[a] < 8 || n[a] > 1024 || n[a] % 2) { msg = "grid sizes must be even and in [8, 1024]"; return PIC_EUNSUPPORTED; }
    if (!factor23(n[a])) { msg = "grid sizes must be of the form 2^a 3^b"; return PIC_EUNSUPPORTED; }
  }
  const double d[3] = {p->dx, p->dy, p->dz};
  for (double x : d)
    if (!(x > 0) || !std::isfinite(x)) { msg = "cell sizes must be positive and finite"; return PIC_EINVAL; }
  const double dmin = std::fmin(p->dx, std::fmin(p->dy, p->dz));
  if (!(p->dt > 0) || !std::isfinite(p->dt) || p->dt > dmin) { msg = "need 0 < c*dt <= min(dx, dy, dz)"; return PIC_EINVAL; }
  if (p->shape_order != 1 && p->shape_order != 3) { msg = "shape_order must be 1 or 3"; return PIC_EUNSUPPORTED; }
  const int nmin = std::min(p->nx, std::min(p->ny, p->nz));
  if (p->center_order < 2 || p->center_order > 32 || p->center_order % 2 || p->center_order > nmin) {
    msg = "center_order must be even, in [2, 32] and <= the smallest grid size";
    return PIC_EUNSUPPORTED;
  }
  if (p->psatd_order != 0 && (p->psatd_order < 2 || p->psatd_order > 64 || p->psatd_order % 2)) {
    msg = "psatd_order must be 0 or even in [2, 64]";
    return PIC_EUNSUPPORTED;
  }
  if (p->dtype != PIC_F32 && p->dtype != PIC_F64) { msg = "dtype must be PIC_F32 or PIC_F64"; return PIC_EINVAL; }
  if (p->flags & ~(uint32_t)(PIC_CURRENT_CORRECTION | PIC_DETERMINISTIC | PIC_SPECTRAL_CENTERING | PIC_NODAL_SOLVER |
                             PIC_KEEP_ORDER | PIC_AVERAGED | PIC_STAGGERED_CYCLE)) {
    msg = "unknown bit in flags";
    return PIC_EINVAL;
  }
  const double vg2 = p->v_gal[0] * p->v_gal[0] + p->v_gal[1] * p->v_gal[1] + p->v_gal[2] * p->v_gal[2];
  if (!std::isfinite(vg2) || vg2 >= 1.0) { msg = "need |v_gal| < c"; return PIC_EINVAL; }
  if ((1.0 + std::sqrt(vg2)) * p->dt > dmin) {  // particles move < 1 cell per step relative to the grid
    msg = "the Galilean frame needs (c + |v_gal|) dt <= min(dx, dy, dz)";
    return PIC_EINVAL;
  }
  if (vg2 > 0 && p->psatd_order == 0) {
    msg = "the Galilean solver needs a finite psatd_order ([k]_c at the Nyquist index)";
    return PIC_EUNSUPPORTED;
  }
  if ((vg2 > 0 || (p->flags & PIC_AVERAGED)) && (p->flags & PIC_CURRENT_CORRECTION)) {
    msg = "PIC_CURRENT_CORRECTION is built for the standard PSATD continuity equation (v_gal = 0, not averaged)";
    return PIC_EUNSUPPORTED;
  }
  if ((p->flags & PIC_CURRENT_CORRECTION) && (p->flags & PIC_NODAL_SOLVER) && p->psatd_order == 0) {
    // [k]_c = k is nonzero at the Nyquist index of an even axis, where the derivative of that
    // self-conjugate mode has no real-valued action (the solver drops it there)
    msg = "PIC_CURRENT_CORRECTION with PIC_NODAL_SOLVER needs a finite psatd_order";
    return PIC_EUNSUPPORTED;
  }
  if (vg2 > 0 && (p->flags & PIC_SPECTRAL_CENTERING)) {
    msg = "PIC_SPECTRAL_CENTERING is built for the standard PSATD update only";
    return PIC_EUNSUPPORTED;
  }
  if ((p->flags & PIC_STAGGERED_CYCLE) &&
      (p->flags & (PIC_NODAL_SOLVER | PIC_SPECTRAL_CENTERING | PIC_AVERAGED))) {
    msg = "PIC_STAGGERED_CYCLE excludes PIC_NODAL_SOLVER, PIC_SPECTRAL_CENTERING and PIC_AVERAGED";
    return PIC_EUNSUPPORTED;
  }
  if ((p->flags & PIC_AVERAGED) && (p->flags & PIC_SPECTRAL_CENTERING)) {
    msg = "PIC_SPECTRAL_CENTERING is built for the standard PSATD update only";
    return PIC_EUNSUPPORTED;
  }
  if ((p->flags & PIC_SPECTRAL_CENTERING) && (p->flags & PIC_NODAL_SOLVER)) {
    msg = "PIC_SPECTRAL_CENTERING and PIC_NODAL_SOLVER exclude each other (the nodal solver has no centering)";
    return PIC_EINVAL;
  }
  return PIC_OK;
}

bool aligned(const void* q) { return (reinterpret_cast<uintptr_t>(q) & 15u) == 0; }

pic_status check_ptr(pic_ctx c, const void* q, const char* name) {
  if (!q) return c->fail(PIC_EINVAL, std::string(name) + " is NULL");
  if (!aligned(q)) return c->fail(PIC_EINVAL, std::string(name) + " is not 16-byte aligned");
  return PIC_OK;
}

pic_status check_species(pic_ctx c, const pic_species* sp, int nsp) {
  if (nsp < 0) return c->fail(PIC_EINVAL, "nsp < 0");
  if (nsp > 0 && !sp) return c->fail(PIC_EINVAL, "species array is NULL");
  for (int s = 0; s < nsp; ++s) {
    const pic_species& x = sp[s];
    if (x.n < 0) return c->fail(PIC_EINVAL, "species n < 0");
    if (x.n > 0x7fffffffLL * 64) return c->fail(PIC_EUNSUPPORTED, "species too large");
    if (!std::isfinite(x.q)) return c->fail(PIC_EINVAL, "species charge must be finite");
    if (!(x.m > 0)) return c->fail(PIC_EINVAL, "species mass must be > 0 (INFINITY for immobile)");
    if (x.n == 0) continue;
    pic_status st;
    if ((st = check_ptr(c, x.cell, "species cell")) != PIC_OK) return st;
    for (int d = 0; d < 3; ++d) {
      if ((st = check_ptr(c, x.off[d], "species off")) != PIC_OK) return st;
      if ((st = check_ptr(c, x.u[d], "species u")) != PIC_OK) return st;
    }
    if (x.w && !aligned(x.w)) return c->fail(PIC_EINVAL, "species w is not 16-byte aligned");
    if (!x.w && !std::isfinite(x.w_const)) return c->fail(PIC_EINVAL, "species w_const must be finite");
  }
  return PIC_OK;
}

template <typename T>
SpeciesView<T> view(const pic_species& x) {
  SpeciesView<T> v{};
  v.n = x.n;
  v.cell = x.cell;
  for (int d = 0; d < 3; ++d) {
    v.off[d] = static_cast<T*>(x.off[d]);
    v.u[d] = static_cast<T*>(x.u[d]);
  }
  v.w = static_cast<T*>(x.w);
  v.w_const = x.w_const;
  v.q = x.q;
  v.m = x.m;
  return v;
}

bool galilean(const pic_params& p) {
  return p.v_gal[0] != 0 || p.v_gal[1] != 0 || p.v_gal[2] != 0 || (p.flags & PIC_AVERAGED) != 0;
}
bool averaged(const pic_params& p) { return (p.flags & PIC_AVERAGED) != 0; }
bool yee_cycle(const pic_params& p) { return (p.flags & PIC_STAGGERED_CYCLE) != 0; }

GridGeom geom(const pic_params& p) {
  GridGeom g = make_geom(p.nx, p.ny, p.nz, p.dx, p.dy, p.dz, p.dt, p.shape_order);
  g.sgx = p.v_gal[0] * p.dt / p.dx;
  g.sgy = p.v_gal[1] * p.dt / p.dy;
  g.sgz = p.v_gal[2] * p.dt / p.dz;
  g.det = (p.flags & PIC_DETERMINISTIC) != 0;
  return g;
}

size_t ncells(const pic_params& p) { return (size_t)p.nx * p.ny * p.nz; }

// ------------------------------------------------------------------ stages

// accumulate: the N2S transposes of E and B add into E_stag / B_stag instead of writing them.
template <typename T>
pic_status do_center(pic_ctx c, int dir, int what, pic_fields* f, bool accumulate = false) {
  Engine<T>& e = static_cast<Engine<T>&>(*c->eng);
  const pic_params& p = c->p;
  const int m = p.center_order / 2;
  const double* cf = c->ccoef.data();
  if (dir == PIC_N2S && what == PIC_J) {
    for (int d = 0; d < 3; ++d)
      center_axis<T>(static_cast<const T*>(f->J_nod[d]), static_cast<T*>(f->J_stag[d]), p.nx, p.ny, p.nz, d, 0, m,
                     cf, c->stream);
  } else if (dir == PIC_S2N && what == PIC_E) {
    for (int d = 0; d < 3; ++d)
      center_axis<T>(static_cast<const T*>(f->E_stag[d]), static_cast<T*>(f->E_nod[d]), p.nx, p.ny, p.nz, d, -1, m,
                     cf, c->stream);
  } else if (dir == PIC_S2N && what == PIC_B) {
    for (int d = 0; d < 3; ++d) {
      const int a0 = (d == 0) ? 1 : 0;
      const int a1 = (d == 2) ? 1 : 2;
      if (a1 == 2 && center_axis_then_z<T>(static_cast<const T*>(f->B_stag[d]), static_cast<T*>(f->B_nod[d]), p.nx,
                                           p.ny, p.nz, a0, -1, m, cf, c->stream))
        continue;  // B^x, B^y: both axes in one pass
      center_axis<T>(static_cast<const T*>(f->B_stag[d]), e.tmp, p.nx, p.ny, p.nz, a0, -1, m, cf, c->stream);
      center_axis<T>(e.tmp, static_cast<T*>(f->B_nod[d]), p.nx, p.ny, p.nz, a1, -1, m, cf, c->stream);
    }
  } else if (dir == PIC_S2N && what == PIC_J) {  // transpose of (N2S, J)
    for (int d = 0; d < 3; ++d)
      center_axis<T>(static_cast<const T*>(f->J_stag[d]), static_cast<T*>(f->J_nod[d]), p.nx, p.ny, p.nz, d, -1, m,
                     cf, c->stream);
  } else if (dir == PIC_N2S && what == PIC_E) {  // transpose of (S2N, E)
    for (int d = 0; d < 3; ++d)
      center_axis<T>(static_cast<const T*>(f->E_nod[d]), static_cast<T*>(f->E_stag[d]), p.nx, p.ny, p.nz, d, 0, m,
                     cf, c->stream, accumulate);
  } else if (dir == PIC_N2S && what == PIC_B) {  // transpose of (S2N, B): the same two axes
    for (int d = 0; d < 3; ++d) {
      const int a0 = (d == 0) ? 1 : 0;
      const int a1 = (d == 2) ? 1 : 2;
      center_axis<T>(static_cast<const T*>(f->B_nod[d]), e.tmp, p.nx, p.ny, p.nz, a1, 0, m, cf, c->stream);
      center_axis<T>(e.tmp, static_cast<T*>(f->B_stag[d]), p.nx, p.ny, p.nz, a0, 0, m, cf, c->stream, accumulate);
    }
  } else {
    return c->fail(PIC_EINVAL, "unsupported (dir, what) pair for pic_center");
  }
  return c->check("pic_center");
}

// The sum of the species' sources without a separate clear: the first species deposited
// overwrites rho_new (starting from rho_static) and, if mobile, J_nod; later ones add.  Each
// deposition sends particles past its tile boxes to the engine's spill arrays, which the
// reduction folds in when that deposition's flag is set.
template <typename T>
struct SourceSum {
  Engine<T>& e;
  const pic_fields* f;
  bool rho_done = false, j_done = false;
  int* flag = nullptr;  // of the current deposition
  SourceSum(Engine<T>& eng, const pic_fields* fields) : e(eng), f(fields) {}
  // rho/J targets of deposit_tiled's direct path, and its flag
  T* spill_rho() { return e.spill[0]; }
  T* const* spill_j() { return e.spill + 1; }
  int* begin() {
    flag = e.spill_flag + (e.dep_k & 1u);
    return flag;
  }
  ReduceArgs<T> reduce_args(bool with_j) {
    ReduceArgs<T> ra;
    ra.acc_mask = (rho_done ? 1 : 0) | (j_done ? 2 : 0);
    ra.base = rho_done ? nullptr : static_cast<const T*>(f->rho_static);
    for (int q = 0; q < 4; ++q) ra.spill[q] = e.spill[q];
    ra.box_faces = e.box_faces;
    ra.rows = 1;  // deposit_tiled's staging layout
    ra.flag = flag;
    ra.next_flag = e.spill_flag + ((e.dep_k + 1u) & 1u);
    ++e.dep_k;
    rho_done = true;
    if (with_j) j_done = true;
    return ra;
  }
  // what no species wrote: rho = rho_static (or zero), J = 0
  void finish(pic_ctx c, bool with_j) {
    const size_t N = ncells(c->p);
    if (!rho_done) {
      if (f->rho_static)
        (void)hipMemcpyAsync(f->rho_new, f->rho_static, N * sizeof(T), hipMemcpyDeviceToDevice, c->stream);
      else
        (void)hipMemsetAsync(f->rho_new, 0, N * sizeof(T), c->stream);
    }
    if (with_j && !j_done)
      for (int d = 0; d < 3; ++d) (void)hipMemsetAsync(f->J_nod[d], 0, N * sizeof(T), c->stream);
  }
};

template <typename T>
void J_ptrs(pic_fields* f, T* J[3]) {
  for (int d = 0; d < 3; ++d) J[d] = static_cast<T*>(f->J_nod[d]);
}

// The staggered cycle's sources: rho^{n+1} on the nodes, J on the Yee grid (J_stag).
template <typename T>
pic_status deposit_yee_all(pic_ctx c, const pic_species* sp, int nsp, pic_fields* f, bool with_j) {
  const size_t N = ncells(c->p);
  if (f->rho_static)
    (void)hipMemcpyAsync(f->rho_new, f->rho_static, N * sizeof(T), hipMemcpyDeviceToDevice, c->stream);
  else
    (void)hipMemsetAsync(f->rho_new, 0, N * sizeof(T), c->stream);
  T* J[3];
  for (int d = 0; d < 3; ++d) {
    J[d] = static_cast<T*>(f->J_stag[d]);
    if (with_j) (void)hipMemsetAsync(J[d], 0, N * sizeof(T), c->stream);
  }
  const GridGeom g = geom(c->p);
  Engine<T>& e = static_cast<Engine<T>&>(*c->eng);
  for (int s = 0; s < nsp; ++s) {
    if (sp[s].n == 0) continue;
    const SpeciesView<T> v = view<T>(sp[s]);
    const bool wj = with_j && std::isfinite(sp[s].m);
    if (e.ensure_species((size_t)s, sp[s].n) != hipSuccess) {  // no scratch: the untiled path
      (void)hipGetLastError();
      // its float atomics add in an order that varies between runs
      if (g.det) return c->fail(PIC_ENOMEM, "pic_deposit: no scratch for the deterministic tiled deposition");
      deposit_yee<T>(g, v, wj, static_cast<T*>(f->rho_new), J, c->stream);
      continue;
    }
    SpeciesScratch<T>& x = e.sps[s];
    tile_sort(g, e.tiles, v.cell, v.n, x.counts[0], x.starts[0], x.cursor, x.dst, c->d_bad, c->stream);
    invert_perm(x.dst, x.perm, v.n, c->stream);
    deposit_yee_tiled<T>(g, e.tiles, v, x.perm, x.starts[0], wj, e.stage, static_cast<T*>(f->rho_new), J, c->stream);
  }
  return PIC_OK;
}

// sort_idx: null = each species' sort indices in the context's species scratch (allocated on
// first use); else 2 n int32 of caller-provided device memory (pic_deposit_noalloc).
template <typename T>
pic_status do_deposit(pic_ctx c, const pic_species* sp, int nsp, pic_fields* f, int mode, int* sort_idx = nullptr) {
  Engine<T>& e = static_cast<Engine<T>&>(*c->eng);
  const bool with_j = (mode == PIC_DEP_RHO_AND_J);
  if (yee_cycle(c->p)) {
    pic_status st = deposit_yee_all<T>(c, sp, nsp, f, with_j);
    if (st != PIC_OK) return st;
    return c->check("pic_deposit");
  }
  T* J[3];
  J_ptrs<T>(f, J);
  SourceSum<T> sum(e, f);
  const GridGeom g = geom(c->p);
  for (int s = 0; s < nsp; ++s) {
    if (sp[s].n == 0) continue;
    int *dst = sort_idx, *perm = sort_idx ? sort_idx + sp[s].n : nullptr;
    if (!sort_idx) {
      hipError_t he = e.ensure_species((size_t)s, sp[s].n);
      if (he != hipSuccess) return c->fail(PIC_ENOMEM, std::string("pic_deposit: ") + hipGetErrorString(he));
      dst = e.sps[s].dst;
      perm = e.sps[s].perm;
    }
    const SpeciesView<T> v = view<T>(sp[s]);
    // visit the caller's particles in tile order through a permutation (caller order untouched)
    tile_sort(g, e.tiles, v.cell, v.n, e.t_counts, e.t_starts, e.t_cursor, dst, c->d_bad, c->stream);
    invert_perm(dst, perm, v.n, c->stream);
    const bool mobile = std::isfinite(sp[s].m);
    int* flag = sum.begin();
    deposit_tiled<T>(g, e.tiles, v, perm, e.t_starts, with_j && mobile, e.stage, c->d_bad, nullptr, nullptr, e.work,
                     sum.spill_rho(), sum.spill_j(), c->stream, flag, e.box_faces);
    deposit_reduce<T>(g, e.tiles, e.t_starts, e.stage, with_j && mobile, static_cast<T*>(f->rho_new), J, c->stream,
                      sum.reduce_args(with_j && mobile));
  }
  sum.finish(c, with_j);
  return c->check("pic_deposit");
}

template <typename T>
void EB_nod(const pic_fields* f, const T* E[3], const T* B[3]) {
  for (int d = 0; d < 3; ++d) {
    E[d] = static_cast<const T*>(f->E_nod[d]);
    B[d] = static_cast<const T*>(f->B_nod[d]);
  }
}

template <typename T>
pic_status do_gather_push(pic_ctx c, const pic_fields* f, pic_species* sp, int nsp) {
  Engine<T>& e = static_cast<Engine<T>&>(*c->eng);
  const GridGeom g = geom(c->p);
  const T *E[3], *B[3];
  EB_nod<T>(f, E, B);
  if (yee_cycle(c->p)) {  // every component from its own Yee positions
    for (int d = 0; d < 3; ++d) {
      E[d] = static_cast<const T*>(f->E_stag[d]);
      B[d] = static_cast<const T*>(f->B_stag[d]);
    }
    for (int s = 0; s < nsp; ++s) gather_push_yee<T>(g, E, B, view<T>(sp[s]), c->stream);
    return c->check("pic_gather_push");
  }
  for (int s = 0; s < nsp; ++s)
    if (std::isfinite(sp[s].m) && sp[s].n > 0) {
      hipError_t he = e.ensure_species((size_t)s, sp[s].n);
      if (he != hipSuccess) return c->fail(PIC_ENOMEM, std::string("pic_gather_push: ") + hipGetErrorString(he));
      SpeciesScratch<T>& x = e.sps[s];
      const SpeciesView<T> v = view<T>(sp[s]);
      // tile order through a permutation; every particle is updated in place
      tile_sort(g, e.tiles, v.cell, v.n, e.t_counts, e.t_starts, e.t_cursor, x.dst, c->d_bad, c->stream);
      invert_perm(x.dst, x.perm, v.n, c->stream);
      gather_push_tiled<T>(g, e.tiles, E, B, v, v, x.perm, e.t_starts, false, nullptr, nullptr, c->stream);
    }
  return c->check("pic_gather_push");
}

template <typename T>
SpeciesView<T> scratch_view(const SpeciesScratch<T>& x, const pic_species& like) {
  SpeciesView<T> v = view<T>(like);
  v.cell = x.cell;
  for (int d = 0; d < 3; ++d) {
    v.off[d] = x.off[d];
    v.u[d] = x.u[d];
  }
  v.w = like.w ? x.w : nullptr;
  return v;
}

template <typename T>
void copy_species(const SpeciesView<T>& from, const SpeciesView<T>& to, hipStream_t st) {
  const size_t n = (size_t)from.n;
  (void)hipMemcpyAsync(to.cell, from.cell, n * sizeof(int32_t), hipMemcpyDeviceToDevice, st);
  for (int d = 0; d < 3; ++d) {
    (void)hipMemcpyAsync(to.off[d], from.off[d], n * sizeof(T), hipMemcpyDeviceToDevice, st);
    (void)hipMemcpyAsync(to.u[d], from.u[d], n * sizeof(T), hipMemcpyDeviceToDevice, st);
  }
  if (from.w) (void)hipMemcpyAsync(to.w, from.w, n * sizeof(T), hipMemcpyDeviceToDevice, st);
}

// forward transforms of the state (E, B) and/or sources (J, rho_old, rho_new)
template <typename T>
void forward_batch(pic_ctx c, Engine<T>& e, const T* const* src, cplx<T>* const* dst, int count,
                   const LineCenter<T>* lc = nullptr) {
  Batch<const T*> in{};
  Batch<cplx<T>*> out{};
  for (int i = 0; i < count; ++i) {
    in.p[i] = src[i];
    out.p[i] = dst[i];
  }
  e.fft.forward(in, out, count, c->stream, lc);
}

// The centering of the real-space cycle as LineCenter of the transforms: J nodes -> Yee (J^d
// along axis d; rho^{n+1}, the fourth array, stays nodal) before the forward transforms, and
// E, B Yee -> nodes (E^d along d, B^d along the two other axes) after the inverse ones.
template <typename T>
LineCenter<T> transform_centering(pic_ctx c, bool to_nodes) {
  LineCenter<T> lc;
  lc.m = (int)c->ccoef.size();
  for (int n = 0; n < lc.m; ++n) lc.c[n] = (T)c->ccoef[n];
  lc.shift = to_nodes ? -1 : 0;
  for (int a = 0; a < 3; ++a) {
    lc.mask[a] = 1u << a;  // E^a (to the nodes) or J^a (to the Yee grid) along axis a
    if (to_nodes) lc.mask[a] |= (7u & ~(1u << a)) << 3;  // B^d, d != a (arrays 3 + d)
  }
  return lc;
}

// The per-mode update, then the inverse transforms: of the staggered state into E_stag,
// B_stag, or (spectral centering) of the nodal spectra the update also wrote, in place in
// the scratch spectra, into E_nod, B_nod.
template <typename T>
void update_and_inverse(pic_ctx c, Engine<T>& e, pic_fields* f, int rho_old_slot, bool spectral = false,
                        bool state_out = true, const LineCenter<T>* to_nodes = nullptr) {
  const pic_params& p = c->p;
  const bool avg = averaged(p);
  {
    StageScope sc(c, ST_UPDATE);
    psatd_update<T>(e.tab, e.Eh, e.Bh, e.Jh, e.rh[rho_old_slot], e.rh[1 - rho_old_slot], p.nx, p.ny, e.fft.nzh,
                    e.fft.pz, spectral ? e.scratch : (avg ? e.Ah : nullptr), c->stream);
  }
  StageScope sc(c, ST_FFT_INV);
  if (avg) {  // the averaged fields of Sec. 4.4 to the Yee grid (the particles' next gather)
    Batch<const cplx<T>*> ain{};
    Batch<cplx<T>*> ascr{};
    Batch<T*> aout{};
    for (int d = 0; d < 3; ++d) {
      ain.p[d] = e.Ah[d];
      ain.p[3 + d] = e.Ah[3 + d];
      aout.p[d] = static_cast<T*>(f->E_avg[d]);
      aout.p[3 + d] = static_cast<T*>(f->B_avg[d]);
    }
    for (int i = 0; i < 6; ++i) ascr.p[i] = e.scratch[i];
    e.fft.inverse(ain, ascr, aout, 6, 1.0 / (double)ncells(p), c->stream);
    if (!state_out) return;  // pic_step: the state stays in Fourier space until the call's end
  }
  Batch<const cplx<T>*> in{};
  Batch<cplx<T>*> scr{};
  Batch<T*> out{};
  const bool nod = spectral || to_nodes;  // (to_nodes: centred to the nodes inside the transforms)
  for (int d = 0; d < 3; ++d) {
    in.p[d] = spectral ? e.scratch[d] : e.Eh[d];
    in.p[3 + d] = spectral ? e.scratch[3 + d] : e.Bh[d];
    out.p[d] = static_cast<T*>(nod ? f->E_nod[d] : f->E_stag[d]);
    out.p[3 + d] = static_cast<T*>(nod ? f->B_nod[d] : f->B_stag[d]);
  }
  for (int i = 0; i < 6; ++i) scr.p[i] = e.scratch[i];
  e.fft.inverse(in, scr, out, 6, 1.0 / (double)ncells(p), c->stream, to_nodes);
}

// The staggered state E_stag, B_stag from the resident spectra (end of a spectral-
// centering pic_step call).
template <typename T>
void state_inverse(pic_ctx c, Engine<T>& e, pic_fields* f) {
  StageScope sc(c, ST_EXIT);
  Batch<const cplx<T>*> in{};
  Batch<cplx<T>*> scr{};
  Batch<T*> out{};
  for (int d = 0; d < 3; ++d) {
    in.p[d] = e.Eh[d];
    in.p[3 + d] = e.Bh[d];
    out.p[d] = static_cast<T*>(f->E_stag[d]);
    out.p[3 + d] = static_cast<T*>(f->B_stag[d]);
  }
  for (int i = 0; i < 6; ++i) scr.p[i] = e.scratch[i];
  e.fft.inverse(in, scr, out, 6, 1.0 / (double)ncells(c->p), c->stream);
}

template <typename T>
pic_status do_push_fields(pic_ctx c, pic_fields* f) {
  Engine<T>& e = static_cast<Engine<T>&>(*c->eng);
  {
    StageScope sc(c, ST_FFT_FWD);
    const T* src[11];
    cplx<T>* dst[11];
    for (int d = 0; d < 3; ++d) {
      src[d] = static_cast<const T*>(f->E_stag[d]);
      dst[d] = e.Eh[d];
      src[3 + d] = static_cast<const T*>(f->B_stag[d]);
      dst[3 + d] = e.Bh[d];
      src[6 + d] = static_cast<const T*>(f->J_stag[d]);
      dst[6 + d] = e.Jh[d];
    }
    src[9] = static_cast<const T*>(f->rho_old);
    dst[9] = e.rh[0];
    src[10] = static_cast<const T*>(f->rho_new);
    dst[10] = e.rh[1];
    forward_batch<T>(c, e, src, dst, 11);
  }
  update_and_inverse<T>(c, e, f, 0);
  return c->check("psatd_push_fields");
}

// Reverse mode of psatd_push_fields: E_stag, B_stag hold the adjoints of the fields at
// n+1 and receive those at n; J_stag, rho_old, rho_new receive the adjoints of the sources.
// The forward map is real-IFFT(M FFT(x)) with a Hermitian-consistent per-mode M, so its
// transpose is the same pipeline with M^H (the 1/N and FFT scalings pair up).
template <typename T>
pic_status do_push_fields_adjoint(pic_ctx c, pic_fields* f) {
  Engine<T>& e = static_cast<Engine<T>&>(*c->eng);
  const pic_params& p = c->p;
  {
    StageScope sc(c, ST_FFT_FWD);
    const T* src[6];
    cplx<T>* dst[6];
    for (int d = 0; d < 3; ++d) {
      src[d] = static_cast<const T*>(f->E_stag[d]);
      dst[d] = e.Eh[d];
      src[3 + d] = static_cast<const T*>(f->B_stag[d]);
      dst[3 + d] = e.Bh[d];
    }
    forward_batch<T>(c, e, src, dst, 6);
  }
  {
    StageScope sc(c, ST_UPDATE);
    psatd_adjoint<T>(e.tab, e.Eh, e.Bh, e.Jh, e.rh[0], e.rh[1], p.nx, p.ny, e.fft.nzh, e.fft.pz, c->stream);
  }
  StageScope sc(c, ST_FFT_INV);
  const double scale = 1.0 / (double)ncells(p);
  Batch<const cplx<T>*> in{};
  Batch<cplx<T>*> scr{};
  Batch<T*> out{};
  for (int d = 0; d < 3; ++d) {
    in.p[d] = e.Eh[d];
    in.p[3 + d] = e.Bh[d];
    out.p[d] = static_cast<T*>(f->E_stag[d]);
    out.p[3 + d] = static_cast<T*>(f->B_stag[d]);
  }
  for (int i = 0; i < 6; ++i) scr.p[i] = e.scratch[i];
  e.fft.inverse(in, scr, out, 6, scale, c->stream);
  // the source adjoints, transformed in place in their own spectra
  cplx<T>* srcs[5] = {e.Jh[0], e.Jh[1], e.Jh[2], e.rh[0], e.rh[1]};
  void* dsts[5] = {f->J_stag[0], f->J_stag[1], f->J_stag[2], f->rho_old, f->rho_new};
  Batch<const cplx<T>*> in2{};
  Batch<cplx<T>*> scr2{};
  Batch<T*> out2{};
  for (int i = 0; i < 5; ++i) {
    in2.p[i] = srcs[i];
    scr2.p[i] = srcs[i];
    out2.p[i] = static_cast<T*>(dsts[i]);
  }
  e.fft.inverse(in2, scr2, out2, 5, scale, c->stream);
  return c->check("psatd_push_fields_adjoint");
}

// pic_step of the fully staggered cycle: gather from the Yee grid, deposit J onto it, no centering.
template <typename T>
pic_status do_step_yee(pic_ctx c, pic_fields* f, pic_species* sp, int nsp, int nsteps) {
  Engine<T>& e = static_cast<Engine<T>&>(*c->eng);
  const pic_params& p = c->p;
  int slot = 0;
  {
    StageScope sc(c, ST_ENTRY);
    const T* src[7];
    cplx<T>* dst[7];
    for (int d = 0; d < 3; ++d) {
      src[d] = static_cast<const T*>(f->E_stag[d]);
      dst[d] = e.Eh[d];
      src[3 + d] = static_cast<const T*>(f->B_stag[d]);
      dst[3 + d] = e.Bh[d];
    }
    src[6] = static_cast<const T*>(f->rho_old);
    dst[6] = e.rh[slot];
    forward_batch<T>(c, e, src, dst, 7);
  }
  const GridGeom g = geom(p);
  const T *E[3], *B[3];
  for (int d = 0; d < 3; ++d) {
    E[d] = static_cast<const T*>(f->E_stag[d]);
    B[d] = static_cast<const T*>(f->B_stag[d]);
  }
  pic_status st;
  for (int q = 0; q < nsp; ++q) {
    hipError_t he = e.ensure_species((size_t)q, sp[q].n);
    if (he != hipSuccess) return c->fail(PIC_ENOMEM, std::string("pic_step: ") + hipGetErrorString(he));
  }
  const size_t N = ncells(p);
  for (int n = 0; n < nsteps; ++n) {
    {
      StageScope sc(c, ST_CLEAR);
      if (f->rho_static)
        (void)hipMemcpyAsync(f->rho_new, f->rho_static, N * sizeof(T), hipMemcpyDeviceToDevice, c->stream);
      else
        (void)hipMemsetAsync(f->rho_new, 0, N * sizeof(T), c->stream);
      for (int d = 0; d < 3; ++d) (void)hipMemsetAsync(f->J_stag[d], 0, N * sizeof(T), c->stream);
    }
    T* J[3] = {static_cast<T*>(f->J_stag[0]), static_cast<T*>(f->J_stag[1]), static_cast<T*>(f->J_stag[2])};
    for (int q = 0; q < nsp; ++q) {
      if (sp[q].n == 0) continue;
      SpeciesScratch<T>& x = e.sps[q];
      const SpeciesView<T> v = view<T>(sp[q]);
      {
        StageScope sc(c, ST_SORT);  // one grouping (cells at n) serves the gather and the deposition
        tile_sort(g, e.tiles, v.cell, v.n, x.counts[0], x.starts[0], x.cursor, x.dst, c->d_bad, c->stream);
        invert_perm(x.dst, x.perm, v.n, c->stream);
      }
      {
        StageScope sc(c, ST_PUSH);
        gather_push_yee_tiled<T>(g, e.tiles, E, B, v, x.perm, x.starts[0], c->stream);
      }
      {
        StageScope sc(c, ST_DEPOSIT);
        deposit_yee_tiled<T>(g, e.tiles, v, x.perm, x.starts[0], std::isfinite(sp[q].m), e.stage,
                             static_cast<T*>(f->rho_new), J, c->stream);
      }
    }
    {
      StageScope sc(c, ST_FFT_FWD);
      const T* src[4] = {static_cast<const T*>(f->J_stag[0]), static_cast<const T*>(f->J_stag[1]),
                         static_cast<const T*>(f->J_stag[2]), static_cast<const T*>(f->rho_new)};
      cplx<T>* dst[4] = {e.Jh[0], e.Jh[1], e.Jh[2], e.rh[1 - slot]};
      forward_batch<T>(c, e, src, dst, 4);
    }
    update_and_inverse<T>(c, e, f, slot);
    slot = 1 - slot;
    if ((st = c->check("pic_step")) != PIC_OK) return st;
  }
  (void)hipMemcpyAsync(f->rho_old, f->rho_new, ncells(p) * sizeof(T), hipMemcpyDeviceToDevice, c->stream);
  return c->check("pic_step");
}

template <typename T>
pic_status do_step(pic_ctx c, pic_fields* f, pic_species* sp, int nsp, int nsteps) {
  Engine<T>& e = static_cast<Engine<T>&>(*c->eng);
  const pic_params& p = c->p;
  if (nsteps == 0) return PIC_OK;
  if (yee_cycle(p)) return do_step_yee<T>(c, f, sp, nsp, nsteps);
  int slot = 0;  // rh[slot] holds rho^n
  {
    StageScope sc(c, ST_ENTRY);
    const T* src[7];
    cplx<T>* dst[7];
    for (int d = 0; d < 3; ++d) {
      src[d] = static_cast<const T*>(f->E_stag[d]);
      dst[d] = e.Eh[d];
      src[3 + d] = static_cast<const T*>(f->B_stag[d]);
      dst[3 + d] = e.Bh[d];
    }
    src[6] = static_cast<const T*>(f->rho_old);
    dst[6] = e.rh[slot];
    forward_batch<T>(c, e, src, dst, 7);
  }
  const GridGeom g = geom(p);
  const bool nodal = (p.flags & PIC_NODAL_SOLVER) != 0;
  const T *Enod[3], *Bnod[3];
  EB_nod<T>(f, Enod, Bnod);
  const bool avg = averaged(p);
  if (nodal)  // nodal solver: the state itself is nodal, gathered directly (averaged: its mean)
    for (int d = 0; d < 3; ++d) {
      Enod[d] = static_cast<const T*>(avg ? f->E_avg[d] : f->E_stag[d]);
      Bnod[d] = static_cast<const T*>(avg ? f->B_avg[d] : f->B_stag[d]);
    }
  T* Jn[3];
  J_ptrs<T>(f, Jn);
  std::vector<char> in_scratch(nsp, 0);
  std::vector<int> layout(nsp, 0);  // which of the species' two groupings describes its current arrays
  for (int q = 0; q < nsp; ++q) {
    hipError_t he = e.ensure_species((size_t)q, sp[q].n);
    if (he != hipSuccess) return c->fail(PIC_ENOMEM, std::string("pic_step: ") + hipGetErrorString(he));
  }
  pic_status st;
  const bool spectral = (p.flags & PIC_SPECTRAL_CENTERING) != 0;
  const bool keep = (p.flags & (PIC_KEEP_ORDER | PIC_DETERMINISTIC)) != 0;
  // Real-space cycle: on every step but the last of the call the centering runs inside the
  // transforms (J_nod -> spectra of J on the Yee grid; updated spectra -> E_nod, B_nod of the
  // next step).  The last step takes the separate passes, so that at return E_stag, B_stag,
  // J_stag and E_nod, B_nod hold what the documented cycle leaves.
  const bool fused = !spectral && !nodal && !avg && e.fft.centering_fusable();
  const LineCenter<T> lc_j = fused ? transform_centering<T>(c, false) : LineCenter<T>();
  const LineCenter<T> lc_eb = fused ? transform_centering<T>(c, true) : LineCenter<T>();
  for (int n = 0; n < nsteps; ++n) {
    const bool mid = fused && n + 1 < nsteps;  // this step's transforms centre
    const bool nod_ready = fused && n > 0;     // E_nod, B_nod from the previous step's inverse
    if (!nodal && (!spectral || n == 0) && !nod_ready) {  // spectral centering: later steps get E_nod, B_nod from the update
      StageScope sc(c, ST_S2N);
      pic_fields t = *f;  // averaged PSATD: the particles see the averaged fields
      if (avg)
        for (int d = 0; d < 3; ++d) {
          t.E_stag[d] = f->E_avg[d];
          t.B_stag[d] = f->B_avg[d];
        }
      if ((st = do_center<T>(c, PIC_S2N, PIC_E, &t)) != PIC_OK) return st;
      if ((st = do_center<T>(c, PIC_S2N, PIC_B, &t)) != PIC_OK) return st;
    }
    SourceSum<T> sum(e, f);
    for (int q = 0; q < nsp; ++q) {
      if (sp[q].n == 0) continue;
      SpeciesScratch<T>& x = e.sps[q];
      if (keep) {  // caller's order: every step visits the particles through a tile permutation
        const SpeciesView<T> v = view<T>(sp[q]);
        const bool mobile = std::isfinite(sp[q].m);
        {
          StageScope sc(c, ST_SORT);
          tile_sort(g, e.tiles, v.cell, v.n, x.counts[0], x.starts[0], x.cursor, x.dst, c->d_bad, c->stream);
          invert_perm(x.dst, x.perm, v.n, c->stream);
        }
        if (mobile) {
          StageScope sc(c, ST_PUSH);
          gather_push_tiled<T>(g, e.tiles, Enod, Bnod, v, v, x.perm, x.starts[0], false, nullptr, nullptr,
                               c->stream);
        }
        {
          StageScope sc(c, ST_DEPOSIT);  // positions moved < 1 cell: the grouping still holds them
          deposit_tiled<T>(g, e.tiles, v, x.perm, x.starts[0], mobile, e.stage, c->d_bad, nullptr, nullptr, e.work,
                           sum.spill_rho(), sum.spill_j(), c->stream, sum.begin(), e.box_faces);
        }
        {
          StageScope sc(c, ST_REDUCE);
          deposit_reduce<T>(g, e.tiles, x.starts[0], e.stage, mobile, static_cast<T*>(f->rho_new), Jn, c->stream,
                            sum.reduce_args(mobile));
        }
        continue;
      }
      const SpeciesView<T> cur = in_scratch[q] ? scratch_view<T>(x, sp[q]) : view<T>(sp[q]);
      const SpeciesView<T> alt = in_scratch[q] ? view<T>(sp[q]) : scratch_view<T>(x, sp[q]);
      const bool mobile = std::isfinite(sp[q].m);
      const size_t nt = (size_t)e.tiles.ntiles;
      // Grouping: on the first step a full counting sort of the caller's order; afterwards
      // the deposition of the previous step has counted the tiles of the current cells.
      const int L = layout[q];
      const bool first = (n == 0);
      {
        StageScope sc(c, ST_SORT);
        if (first) {
          tile_sort(g, e.tiles, cur.cell, cur.n, x.counts[0], x.starts[0], x.cursor, x.dst, c->d_bad, c->stream);
          invert_perm(x.dst, x.perm, cur.n, c->stream);
        } else if (mobile) {
          scan_counts(e.tiles, x.counts[1 - L], x.starts[1 - L], x.cursor, c->stream);
          neighbour_bases(e.tiles, x.starts[L], x.nbr, x.starts[1 - L], x.nbr_base, x.cursor, c->stream);
        }
        if (mobile) (void)hipMemsetAsync(x.counts[first ? 1 : L], 0, sizeof(int) * (nt + 1), c->stream);
      }
      const int* dep_starts = first ? x.starts[0] : (mobile ? x.starts[1 - L] : x.starts[L]);
      {
        StageScope sc(c, ST_PUSH);
        if (first && mobile)
          gather_push_tiled<T>(g, e.tiles, Enod, Bnod, cur, alt, x.perm, x.starts[0], true, nullptr, nullptr,
                               c->stream);
        else if (first)
          permute_species<T>(cur, alt, x.dst, c->stream);
        else if (mobile)
          gather_push_tiled<T>(g, e.tiles, Enod, Bnod, cur, alt, nullptr, x.starts[L], true, x.cursor, x.nbr_base,
                               c->stream);
      }
      const SpeciesView<T> dep = (first || mobile) ? alt : cur;  // immobile species stay put after the first step
      {
        StageScope sc(c, ST_DEPOSIT);
        int* nextc = mobile ? x.counts[first ? 1 : L] : nullptr;
        deposit_tiled<T>(g, e.tiles, dep, nullptr, dep_starts, mobile, e.stage, c->d_bad, nextc,
                         mobile ? x.nbr : nullptr, e.work, sum.spill_rho(), sum.spill_j(), c->stream, sum.begin(),
                         e.box_faces);
      }
      {
        StageScope sc(c, ST_REDUCE);
        deposit_reduce<T>(g, e.tiles, dep_starts, e.stage, mobile, static_cast<T*>(f->rho_new), Jn, c->stream,
                          sum.reduce_args(mobile));
      }
      if (first || mobile) in_scratch[q] = !in_scratch[q];
      // layout index of the grouping the particles are now in
      if (mobile) layout[q] = first ? 0 : 1 - L;
    }
    {
      StageScope sc(c, ST_CLEAR);
      sum.finish(c, true);
    }
    if (!spectral && !nodal && !mid) {
      StageScope sc(c, ST_N2S);
      if ((st = do_center<T>(c, PIC_N2S, PIC_J, f)) != PIC_OK) return st;
    }
    {
      StageScope sc(c, ST_FFT_FWD);
      // spectral centering: the update centres J; nodal solver: J stays on the nodes; mid: the
      // forward transforms centre J
      void* const* J = (spectral || nodal || mid) ? f->J_nod : f->J_stag;
      const T* src[4] = {static_cast<const T*>(J[0]), static_cast<const T*>(J[1]), static_cast<const T*>(J[2]),
                         static_cast<const T*>(f->rho_new)};
      cplx<T>* dst[4] = {e.Jh[0], e.Jh[1], e.Jh[2], e.rh[1 - slot]};
      forward_batch<T>(c, e, src, dst, 4, mid ? &lc_j : nullptr);
    }
    update_and_inverse<T>(c, e, f, slot, spectral, !avg, mid ? &lc_eb : nullptr);
    slot = 1 - slot;
    if ((st = c->check("pic_step")) != PIC_OK) return st;
  }
  if (avg) state_inverse<T>(c, e, f);  // averaged: the particles used E_avg, B_avg; the state once, here
  if (spectral) {  // the outputs the real-space cycle leaves: the staggered state and J_stag
    state_inverse<T>(c, e, f);
    StageScope sc(c, ST_N2S);
    if ((st = do_center<T>(c, PIC_N2S, PIC_J, f)) != PIC_OK) return st;
  }
  // particles left in the scratch arrays go back to the caller's arrays (tile order kept)
  for (int q = 0; q < nsp; ++q)
    if (in_scratch[q] && sp[q].n > 0) copy_species<T>(scratch_view<T>(e.sps[q], sp[q]), view<T>(sp[q]), c->stream);
  (void)hipMemcpyAsync(f->rho_old, f->rho_new, ncells(p) * sizeof(T), hipMemcpyDeviceToDevice, c->stream);
  return c->check("pic_step");
}

// Reverse mode of one pic_step step (see pic_step_adjoint in pic.h).
template <typename T>
pic_status do_step_adjoint(pic_ctx c, pic_fields* f, const pic_species* sp, int nsp, pic_fields* a,
                           const pic_species_adjoint* asp) {
  Engine<T>& e = static_cast<Engine<T>&>(*c->eng);
  const pic_params& p = c->p;
  const size_t N = ncells(p);
  const GridGeom g = geom(p);
  const bool nodal = (p.flags & PIC_NODAL_SOLVER) != 0;
  pic_status st;
  // nodal fields of the state at n (the nodal solver gathers its state directly)
  const T* F[6];
  for (int d = 0; d < 3; ++d) {
    F[d] = static_cast<const T*>(nodal ? f->E_stag[d] : f->E_nod[d]);
    F[3 + d] = static_cast<const T*>(nodal ? f->B_stag[d] : f->B_nod[d]);
  }
  if (!nodal) {
    StageScope sc(c, ST_S2N);
    if ((st = do_center<T>(c, PIC_S2N, PIC_E, f)) != PIC_OK) return st;
    if ((st = do_center<T>(c, PIC_S2N, PIC_B, f)) != PIC_OK) return st;
  }
  // field solve: a->E_stag, a->B_stag in place; dL/dJ into J_stag (nodal solver: J_nod),
  // dL/drho^n into rho_old, the field solve's dL/drho^{n+1} into E_nod[0] (then added to
  // the carried adjoint of rho^{n+1} in rho_new)
  {
    pic_fields t = *a;
    t.rho_new = a->E_nod[0];
    if (nodal)
      for (int d = 0; d < 3; ++d) t.J_stag[d] = a->J_nod[d];
    if ((st = do_push_fields_adjoint<T>(c, &t)) != PIC_OK) return st;
  }
  add_into<T>(static_cast<T*>(a->rho_new), static_cast<const T*>(a->E_nod[0]), (int64_t)N, c->stream);
  if (!nodal) {
    StageScope sc(c, ST_N2S);
    if ((st = do_center<T>(c, PIC_S2N, PIC_J, a)) != PIC_OK) return st;  // J_stag -> J_nod (transpose of N2S)
  }
  {
    Batch<T*> z{};
    for (int d = 0; d < 3; ++d) {
      z.p[d] = static_cast<T*>(a->E_nod[d]);
      z.p[3 + d] = static_cast<T*>(a->B_nod[d]);
    }
    zero_arrays<T>(z, 6, (int64_t)N, c->stream);
  }
  const T* L[4] = {static_cast<const T*>(a->rho_new), static_cast<const T*>(a->J_nod[0]),
                   static_cast<const T*>(a->J_nod[1]), static_cast<const T*>(a->J_nod[2])};
  T* out[6];
  for (int d = 0; d < 3; ++d) {
    out[d] = static_cast<T*>(a->E_nod[d]);
    out[3 + d] = static_cast<T*>(a->B_nod[d]);
  }
  for (int q = 0; q < nsp; ++q) {
    if (sp[q].n == 0) continue;
    hipError_t he = e.ensure_species((size_t)q, sp[q].n);
    if (he == hipSuccess && !e.astage) {
      const size_t B = (size_t)deposit_box(p.shape_order);
      he = e.alloc(&e.astage, (size_t)e.tiles.ntiles * 6 * B * B * B);
    }
    if (he != hipSuccess) return c->fail(PIC_ENOMEM, std::string("pic_step_adjoint: ") + hipGetErrorString(he));
    SpeciesScratch<T>& x = e.sps[q];
    const SpeciesView<T> v = view<T>(sp[q]);
    {
      StageScope sc(c, ST_SORT);
      tile_sort(g, e.tiles, v.cell, v.n, x.counts[0], x.starts[0], x.cursor, x.dst, c->d_bad, c->stream);
      invert_perm(x.dst, x.perm, v.n, c->stream);
    }
    Batch<T*> lam{}, lamF{};
    for (int d = 0; d < 3; ++d) {
      lam.p[d] = static_cast<T*>(asp[q].off[d]);
      lam.p[3 + d] = static_cast<T*>(asp[q].u[d]);
      lamF.p[d] = x.off[d];  // the species scratch holds dL/d(E_p, B_p)
      lamF.p[3 + d] = x.u[d];
    }
    {
      StageScope sc(c, ST_PUSH);
      particle_adjoint<T>(g, e.tiles, v, lam, x.perm, x.starts[0], F, L, lamF, c->stream);
    }
    if (std::isfinite(sp[q].m)) {
      StageScope sc(c, ST_DEPOSIT);
      const T* val[6] = {x.off[0], x.off[1], x.off[2], x.u[0], x.u[1], x.u[2]};
      scatter_tiled<T>(g, e.tiles, v, x.perm, x.starts[0], val, out, e.astage, c->stream);
    }
  }
  // the gathered fields' adjoints back to the state grid, added to the field solve's
  if (nodal) {
    for (int d = 0; d < 3; ++d) {
      add_into<T>(static_cast<T*>(a->E_stag[d]), out[d], (int64_t)N, c->stream);
      add_into<T>(static_cast<T*>(a->B_stag[d]), out[3 + d], (int64_t)N, c->stream);
    }
  } else {
    StageScope sc(c, ST_S2N);
    pic_fields t{};
    for (int d = 0; d < 3; ++d) {  // the transposed centering adds straight into the state's adjoint
      t.E_nod[d] = a->E_nod[d];
      t.B_nod[d] = a->B_nod[d];
      t.E_stag[d] = a->E_stag[d];
      t.B_stag[d] = a->B_stag[d];
    }
    if ((st = do_center<T>(c, PIC_N2S, PIC_E, &t, true)) != PIC_OK) return st;
    if ((st = do_center<T>(c, PIC_N2S, PIC_B, &t, true)) != PIC_OK) return st;
  }
  return c->check("pic_step_adjoint");
}

// Gauss's law (continuity = false: E_stag, rho_old) or the continuity equation (continuity =
// true: J, rho_old = rho^n, rho_new = rho^{n+1}) in Fourier space; *out = ||r|| / ||source||.
template <typename T>
pic_status do_div_residual(pic_ctx c, const pic_fields* f, double* out, bool continuity) {
  Engine<T>& e = static_cast<Engine<T>&>(*c->eng);
  const pic_params& p = c->p;
  const bool nodal = (p.flags & PIC_NODAL_SOLVER) != 0;
  const char* where = continuity ? "pic_continuity_residual" : "pic_gauss_residual";
  const T* src[5];
  for (int d = 0; d < 3; ++d)
    src[d] = static_cast<const T*>(continuity ? (nodal ? f->J_nod[d] : f->J_stag[d]) : f->E_stag[d]);
  src[3] = static_cast<const T*>(continuity ? f->rho_new : f->rho_old);
  src[4] = static_cast<const T*>(f->rho_old);
  cplx<T>* dst[5] = {e.scratch[0], e.scratch[1], e.scratch[2], e.scratch[3], e.scratch[4]};
  forward_batch<T>(c, e, src, dst, continuity ? 5 : 4);
  (void)hipMemsetAsync(c->d_acc, 0, 2 * sizeof(double), c->stream);
  const cplx<T>* V[3] = {e.scratch[0], e.scratch[1], e.scratch[2]};
  if (continuity)
    div_residual<T>(e.tab, V, e.scratch[3], 1.0 / p.dt, e.scratch[4], -1.0 / p.dt, p.nx, p.ny, e.fft.nzh, e.fft.pz,
                    p.nz, c->d_acc, c->stream);
  else
    div_residual<T>(e.tab, V, e.scratch[3], -1.0, nullptr, 0.0, p.nx, p.ny, e.fft.nzh, e.fft.pz, p.nz, c->d_acc,
                    c->stream);
  double h[2];
  hipError_t he = hipMemcpyAsync(h, c->d_acc, sizeof(h), hipMemcpyDeviceToHost, c->stream);
  if (he == hipSuccess) he = hipStreamSynchronize(c->stream);
  if (he != hipSuccess) return c->fail(PIC_EHIP, std::string(where) + ": " + hipGetErrorString(he));
  out[0] = h[1] > 0 ? std::sqrt(h[0] / h[1]) : std::sqrt(h[0]);
  return c->check(where);
}

template <typename T>
pic_status do_diag(pic_ctx c, const pic_fields* f, double out[2]) {
  const pic_params& p = c->p;
  const size_t N = ncells(p);
  (void)hipMemsetAsync(c->d_acc, 0, 2 * sizeof(double), c->stream);
  Batch<const T*> a{};
  for (int d = 0; d < 3; ++d) {
    a.p[d] = static_cast<const T*>(f->E_stag[d]);
    a.p[3 + d] = static_cast<const T*>(f->B_stag[d]);
  }
  sum_squares<T>(a, 6, (int64_t)N, c->d_acc, c->stream);
  sum_plain<T>(static_cast<const T*>(f->rho_old), (int64_t)N, c->d_acc + 1, c->stream);
  double h[2];
  hipError_t e = hipMemcpyAsync(h, c->d_acc, sizeof(h), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return c->fail(PIC_EHIP, std::string("pic_diagnostics: ") + hipGetErrorString(e));
  const double dV = p.dx * p.dy * p.dz;
  out[0] = 0.5 * h[0] * dV;
  out[1] = h[1] * dV;
  return PIC_OK;
}

pic_status check_fields(pic_ctx c, const pic_fields* f, bool E_stag, bool B_stag, bool E_nod, bool B_nod, bool J_nod,
                        bool J_stag, bool rho_old, bool rho_new) {
  if (!f) return c->fail(PIC_EINVAL, "fields is NULL");
  pic_status st;
  for (int d = 0; d < 3; ++d) {
    if (E_stag && (st = check_ptr(c, f->E_stag[d], "E_stag")) != PIC_OK) return st;
    if (B_stag && (st = check_ptr(c, f->B_stag[d], "B_stag")) != PIC_OK) return st;
    if (E_nod && (st = check_ptr(c, f->E_nod[d], "E_nod")) != PIC_OK) return st;
    if (B_nod && (st = check_ptr(c, f->B_nod[d], "B_nod")) != PIC_OK) return st;
    if (J_nod && (st = check_ptr(c, f->J_nod[d], "J_nod")) != PIC_OK) return st;
    if (J_stag && (st = check_ptr(c, f->J_stag[d], "J_stag")) != PIC_OK) return st;
  }
  if (rho_old && (st = check_ptr(c, f->rho_old, "rho_old")) != PIC_OK) return st;
  if (rho_new && (st = check_ptr(c, f->rho_new, "rho_new")) != PIC_OK) return st;
  if (f->rho_static && !aligned(f->rho_static)) return c->fail(PIC_EINVAL, "rho_static is not 16-byte aligned");
  return PIC_OK;
}

pic_status check_avg(pic_ctx c, const pic_fields* f) {
  if (!averaged(c->p)) return PIC_OK;
  pic_status st;
  for (int d = 0; d < 3; ++d) {
    if ((st = check_ptr(c, f->E_avg[d], "E_avg")) != PIC_OK) return st;
    if ((st = check_ptr(c, f->B_avg[d], "B_avg")) != PIC_OK) return st;
  }
  return PIC_OK;
}

pic_status device_ok(pic_ctx c) {
  if (!c) return PIC_ESTATE;
  if (!c->eng) return c->fail(PIC_ESTATE, "context has no engine");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != c->device) (void)hipSetDevice(c->device);
  return PIC_OK;
}

}  // namespace

#define PIC_DISPATCH(ctx, fn, ...) \
  ((ctx)->p.dtype == PIC_F32 ? fn<float>(ctx, __VA_ARGS__) : fn<double>(ctx, __VA_ARGS__))

extern "C" {

pic_status pic_init(const pic_params* p, void* hip_stream, pic_ctx* out) {
  if (!out) {
    g_init_error = "out is NULL";
    return PIC_EINVAL;
  }
  *out = nullptr;
  std::string msg;
  pic_status st = validate_params(p, msg);
  if (st != PIC_OK) {
    g_init_error = msg;
    return st;
  }
  auto c = std::make_unique<pic_ctx_s>();
  c->p = *p;
  c->stream = static_cast<hipStream_t>(hip_stream);
  if (hipGetDevice(&c->device) != hipSuccess) {
    g_init_error = "no HIP device";
    return PIC_EHIP;
  }
  // this device's copy of the no-allocation scratch (an error is reported by pic_deposit_noalloc)
  c->noalloc = scratch_address(c->device, c->noalloc_err);
  const int m = p->center_order / 2;
  c->ccoef.resize(m);
  alpha_staggered(m, c->ccoef.data());
  for (double& a : c->ccoef) a *= 0.5;
  hipError_t e;
  if (p->dtype == PIC_F32) {
    auto eng = std::make_unique<Engine<float>>();
    e = build_engine<float>(*p, *eng);
    c->eng = std::move(eng);
  } else {
    auto eng = std::make_unique<Engine<double>>();
    e = build_engine<double>(*p, *eng);
    c->eng = std::move(eng);
  }
  if (e == hipSuccess) e = hipMalloc(&c->d_acc, 2 * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&c->d_bad, sizeof(int));
  if (e == hipSuccess) e = hipMemset(c->d_bad, 0, sizeof(int));
  if (e != hipSuccess) {
    g_init_error = std::string("pic_init: ") + hipGetErrorString(e);
    (void)hipGetLastError();
    return (e == hipErrorOutOfMemory) ? PIC_ENOMEM : PIC_EHIP;
  }
  *out = c.release();
  return PIC_OK;
}

pic_status pic_destroy(pic_ctx ctx) {
  if (!ctx) return PIC_EINVAL;
  (void)hipStreamSynchronize(ctx->stream);
  ctx->collect();
  for (auto& ev : ctx->pool) {
    (void)hipEventDestroy(ev.a);
    (void)hipEventDestroy(ev.b);
  }
  if (ctx->d_acc) (void)hipFree(ctx->d_acc);
  if (ctx->d_bad) (void)hipFree(ctx->d_bad);
  ctx->eng.reset();
  delete ctx;
  return PIC_OK;
}

pic_status pic_set_stream(pic_ctx ctx, void* hip_stream) {
  if (!ctx) return PIC_EINVAL;
  ctx->stream = static_cast<hipStream_t>(hip_stream);
  return PIC_OK;
}

pic_status pic_deposit(pic_ctx ctx, const pic_species* sp, int nsp, pic_fields* f, int mode) {
  pic_status st = device_ok(ctx);
  if (st != PIC_OK) return st;
  if (mode != PIC_DEP_RHO_AND_J && mode != PIC_DEP_RHO_ONLY) return ctx->fail(PIC_EINVAL, "bad deposit mode");
  if ((st = check_species(ctx, sp, nsp)) != PIC_OK) return st;
  const bool wj = mode == PIC_DEP_RHO_AND_J, yee = yee_cycle(ctx->p);  // staggered cycle: J into J_stag
  if ((st = check_fields(ctx, f, false, false, false, false, wj && !yee, wj && yee, false, true)) != PIC_OK)
    return st;
  return PIC_DISPATCH(ctx, do_deposit, sp, nsp, f, mode);
}

pic_status pic_deposit_noalloc(pic_ctx ctx, const pic_species* sp, int nsp, pic_fields* f, int mode) {
  pic_status st = device_ok(ctx);
  if (st != PIC_OK) return st;
  if (mode != PIC_DEP_RHO_AND_J && mode != PIC_DEP_RHO_ONLY) return ctx->fail(PIC_EINVAL, "bad deposit mode");
  if (yee_cycle(ctx->p))
    return ctx->fail(PIC_EUNSUPPORTED, "pic_deposit_noalloc: not with PIC_STAGGERED_CYCLE");
  if ((st = check_species(ctx, sp, nsp)) != PIC_OK) return st;
  for (int s = 0; s < nsp; ++s)
    if (sp[s].n > kNoAllocMaxParticles)
      return ctx->fail(PIC_EUNSUPPORTED, "pic_deposit_noalloc: more than " + std::to_string(kNoAllocMaxParticles) +
                                             " particles in one species (the size of its static scratch)");
  if (!ctx->noalloc) return ctx->fail(PIC_EHIP, "pic_deposit_noalloc: " + ctx->noalloc_err);
  const bool wj = mode == PIC_DEP_RHO_AND_J;
  if ((st = check_fields(ctx, f, false, false, false, false, wj, false, false, true)) != PIC_OK) return st;
  return PIC_DISPATCH(ctx, do_deposit, sp, nsp, f, mode, static_cast<int*>(ctx->noalloc));
}

pic_status pic_center(pic_ctx ctx, int dir, int what, pic_fields* f) {
  pic_status st = device_ok(ctx);
  if (st != PIC_OK) return st;
  if (!f) return ctx->fail(PIC_EINVAL, "fields is NULL");
  if ((dir != PIC_N2S && dir != PIC_S2N) || (what != PIC_J && what != PIC_E && what != PIC_B))
    return ctx->fail(PIC_EINVAL, "unsupported (dir, what) pair for pic_center");
  if (what == PIC_J)
    st = check_fields(ctx, f, false, false, false, false, true, true, false, false);
  else if (what == PIC_E)
    st = check_fields(ctx, f, true, false, true, false, false, false, false, false);
  else
    st = check_fields(ctx, f, false, true, false, true, false, false, false, false);
  if (st != PIC_OK) return st;
  return PIC_DISPATCH(ctx, do_center, dir, what, f);
}

pic_status psatd_push_fields(pic_ctx ctx, pic_fields* f) {
  pic_status st = device_ok(ctx);
  if (st != PIC_OK) return st;
  if ((st = check_fields(ctx, f, true, true, false, false, false, true, true, true)) != PIC_OK) return st;
  if ((st = check_avg(ctx, f)) != PIC_OK) return st;
  return PIC_DISPATCH(ctx, do_push_fields, f);
}

pic_status psatd_push_fields_adjoint(pic_ctx ctx, pic_fields* f) {
  pic_status st = device_ok(ctx);
  if (st != PIC_OK) return st;
  if (galilean(ctx->p)) return ctx->fail(PIC_EUNSUPPORTED, "no reverse mode for the Galilean solver");
  if ((st = check_fields(ctx, f, true, true, false, false, false, true, true, true)) != PIC_OK) return st;
  return PIC_DISPATCH(ctx, do_push_fields_adjoint, f);
}

pic_status pic_gather_push(pic_ctx ctx, const pic_fields* f, pic_species* sp, int nsp) {
  pic_status st = device_ok(ctx);
  if (st != PIC_OK) return st;
  if ((st = check_species(ctx, sp, nsp)) != PIC_OK) return st;
  const bool yee = yee_cycle(ctx->p);  // the staggered cycle gathers from the Yee-grid arrays
  if ((st = check_fields(ctx, f, yee, yee, !yee, !yee, false, false, false, false)) != PIC_OK) return st;
  return PIC_DISPATCH(ctx, do_gather_push, f, sp, nsp);
}

pic_status pic_step(pic_ctx ctx, pic_fields* f, pic_species* sp, int nsp, int nsteps) {
  pic_status st = device_ok(ctx);
  if (st != PIC_OK) return st;
  if (nsteps < 0) return ctx->fail(PIC_EINVAL, "nsteps < 0");
  if ((st = check_species(ctx, sp, nsp)) != PIC_OK) return st;
  if ((st = check_fields(ctx, f, true, true, true, true, true, true, true, true)) != PIC_OK) return st;
  if ((st = check_avg(ctx, f)) != PIC_OK) return st;
  return PIC_DISPATCH(ctx, do_step, f, sp, nsp, nsteps);
}

pic_status pic_step_adjoint(pic_ctx ctx, pic_fields* f, const pic_species* sp, int nsp, pic_fields* adj,
                            const pic_species_adjoint* asp) {
  pic_status st = device_ok(ctx);
  if (st != PIC_OK) return st;
  if (galilean(ctx->p)) return ctx->fail(PIC_EUNSUPPORTED, "no reverse mode for the Galilean solver");
  if (yee_cycle(ctx->p)) return ctx->fail(PIC_EUNSUPPORTED, "no reverse mode for the staggered cycle");
  if ((st = check_species(ctx, sp, nsp)) != PIC_OK) return st;
  const bool nodal = (ctx->p.flags & PIC_NODAL_SOLVER) != 0;
  if ((st = check_fields(ctx, f, true, true, !nodal, !nodal, false, false, false, false)) != PIC_OK) return st;
  if ((st = check_fields(ctx, adj, true, true, true, true, true, true, true, true)) != PIC_OK) return st;
  if (nsp > 0 && !asp) return ctx->fail(PIC_EINVAL, "species adjoint array is NULL");
  for (int q = 0; q < nsp; ++q) {
    if (sp[q].n == 0) continue;
    for (int d = 0; d < 3; ++d) {
      if ((st = check_ptr(ctx, asp[q].off[d], "adjoint off")) != PIC_OK) return st;
      if ((st = check_ptr(ctx, asp[q].u[d], "adjoint u")) != PIC_OK) return st;
    }
  }
  return PIC_DISPATCH(ctx, do_step_adjoint, f, sp, nsp, adj, asp);
}

pic_status pic_sync(pic_ctx ctx) {
  if (!ctx) return PIC_EINVAL;
  hipError_t e = hipStreamSynchronize(ctx->stream);
  if (e == hipSuccess) e = hipGetLastError();
  int bad = 0;
  if (e == hipSuccess) e = hipMemcpy(&bad, ctx->d_bad, sizeof(int), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return ctx->fail(PIC_EHIP, std::string("pic_sync: ") + hipGetErrorString(e));
  if (bad != 0) {
    (void)hipMemset(ctx->d_bad, 0, sizeof(int));
    return ctx->fail(PIC_EINVAL, "pic_sync: " + std::to_string(bad) +
                                     " particle(s) had an out-of-range cell index and were skipped");
  }
  return PIC_OK;
}

pic_status pic_diagnostics(pic_ctx ctx, const pic_fields* f, double out[2]) {
  pic_status st = device_ok(ctx);
  if (st != PIC_OK) return st;
  if (!out) return ctx->fail(PIC_EINVAL, "out is NULL");
  if ((st = check_fields(ctx, f, true, true, false, false, false, false, true, false)) != PIC_OK) return st;
  return PIC_DISPATCH(ctx, do_diag, f, out);
}

pic_status pic_gauss_residual(pic_ctx ctx, const pic_fields* f, double* out) {
  pic_status st = device_ok(ctx);
  if (st != PIC_OK) return st;
  if (!out) return ctx->fail(PIC_EINVAL, "out is NULL");
  if ((st = check_fields(ctx, f, true, false, false, false, false, false, true, false)) != PIC_OK) return st;
  return PIC_DISPATCH(ctx, do_div_residual, f, out, false);
}

pic_status pic_continuity_residual(pic_ctx ctx, const pic_fields* f, double* out) {
  pic_status st = device_ok(ctx);
  if (st != PIC_OK) return st;
  if (!out) return ctx->fail(PIC_EINVAL, "out is NULL");
  const bool nodal = (ctx->p.flags & PIC_NODAL_SOLVER) != 0;
  if ((st = check_fields(ctx, f, false, false, false, false, nodal, !nodal, true, true)) != PIC_OK) return st;
  return PIC_DISPATCH(ctx, do_div_residual, f, out, true);
}

pic_status pic_profile(pic_ctx ctx, int enable) {
  if (!ctx) return PIC_EINVAL;
  ctx->profiling = enable != 0;
  return PIC_OK;
}

pic_status pic_stage_times(pic_ctx ctx, double* ms, int64_t* count, int nstage) {
  if (!ctx) return PIC_EINVAL;
  if ((nstage > 0 && (!ms || !count)) || nstage < 0) return ctx->fail(PIC_EINVAL, "bad output arrays");
  ctx->collect();
  for (int s = 0; s < nstage && s < kNumStages; ++s) {
    ms[s] = ctx->stage_ms[s];
    count[s] = ctx->stage_count[s];
  }
  for (int s = 0; s < kNumStages; ++s) {
    ctx->stage_ms[s] = 0;
    ctx->stage_count[s] = 0;
  }
  return PIC_OK;
}

const char* pic_stage_name(int s) { return (s >= 0 && s < kNumStages) ? kStageNames[s] : "unknown"; }
int pic_num_stages(void) { return kNumStages; }

const char* pic_last_error(pic_ctx ctx) { return ctx ? ctx->err.c_str() : g_init_error.c_str(); }

// ------------------------------------------------------------------ closed-form diagnostics (host)

pic_status pic_modified_wavenumber(int32_t n, double d, int32_t order, int32_t kind, double* out) {
  if (!out || n < 2 || !(d > 0) || order < 0 || order > 64 || order % 2 || (kind != 0 && kind != 1)) {
    g_init_error = "pic_modified_wavenumber: need n >= 2, d > 0, order even in [0, 64], kind 0 or 1, out";
    return PIC_EINVAL;
  }
  if (kind == 0)
    k_staggered_axis(n, d, order, out);
  else
    k_centered_axis(n, d, order, out);
  return PIC_OK;
}

pic_status pic_centering_factor(int32_t n, int32_t center_order, double* out) {
  if (!out || n < 2 || center_order < 2 || center_order > 64 || center_order % 2) {
    g_init_error = "pic_centering_factor: need n >= 2, center_order even in [2, 64], out";
    return PIC_EINVAL;
  }
  const int m = center_order / 2;
  std::vector<double> a(m);
  alpha_staggered(m, a.data());
  const double two_pi = 6.283185307179586476925286766559;
  for (int i = 0; i < n; ++i) {
    const int f = (i <= (n - 1) / 2) ? i : i - n;
    const double kd = two_pi * f / n;
    long double z = 0.0L;
    for (int q = 1; q <= m; ++q) z += (long double)a[q - 1] * std::cos(kd * (q - 0.5));
    out[i] = (double)z;
  }
  return PIC_OK;
}

pic_status pic_stencil_extent(const pic_params* p, int32_t axis, int32_t coefficient, double* out) {
  std::string msg;
  pic_status st = validate_params(p, msg);
  if (st != PIC_OK) {
    g_init_error = "pic_stencil_extent: " + msg;
    return st;
  }
  if (!out || axis < 0 || axis > 2 || coefficient < 0 || coefficient > 4) {
    g_init_error = "pic_stencil_extent: need axis in 0..2, coefficient in 0..4 (C, S/w, X1, X2, X3), out";
    return PIC_EINVAL;
  }
  const int n[3] = {p->nx, p->ny, p->nz};
  const double d[3] = {p->dx, p->dy, p->dz};
  const bool nodal = (p->flags & PIC_NODAL_SOLVER) != 0;
  std::vector<double> ks[3];
  for (int a = 0; a < 3; ++a) {
    ks[a].resize(n[a]);
    if (nodal)
      k_centered_axis(n[a], d[a], p->psatd_order, ks[a].data());
    else
      k_staggered_axis(n[a], d[a], p->psatd_order, ks[a].data());
  }
  // g averaged over the two other axes (full spectrum), per index along ``axis``
  const int b = (axis + 1) % 3, c = (axis + 2) % 3;
  std::vector<double> gavg(n[axis], 0.0);
  for (int i = 0; i < n[axis]; ++i) {
    long double acc = 0.0L;
    for (int j = 0; j < n[b]; ++j)
      for (int k = 0; k < n[c]; ++k) {
        const double w = std::sqrt(ks[axis][i] * ks[axis][i] + ks[b][j] * ks[b][j] + ks[c][k] * ks[c][k]);
        double v[5];
        psatd_coefficients(w, p->dt, &v[0], &v[1], &v[2], &v[3], &v[4]);
        acc += v[coefficient];
      }
    gavg[i] = (double)(acc / ((long double)n[b] * n[c]));
  }
  // inverse DFT along ``axis``: Gamma(x_j) = | (1/n) sum_i g(k_i) exp(+i k_i x_j) |
  const double two_pi = 6.283185307179586476925286766559;
  for (int j = 0; j < n[axis]; ++j) {
    long double re = 0.0L, im = 0.0L;
    for (int i = 0; i < n[axis]; ++i) {
      const double ph = two_pi * (double)(((long long)i * j) % n[axis]) / n[axis];
      re += gavg[i] * std::cos(ph);
      im += gavg[i] * std::sin(ph);
    }
    out[j] = (double)(std::sqrt(re * re + im * im) / n[axis]);
  }
  return PIC_OK;
}

const char* pic_strerror(pic_status s) {
  switch (s) {
    case PIC_OK: return "success";
    case PIC_EINVAL: return "invalid argument";
    case PIC_EUNSUPPORTED: return "unsupported configuration";
    case PIC_EHIP: return "HIP error";
    case PIC_ENOMEM: return "out of device memory";
    case PIC_ESTATE: return "invalid state";
  }
  return "unknown status";
}

}  // extern "C"
