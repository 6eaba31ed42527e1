/*
 * pic.h -- C ABI of the hybrid nodal-staggered PSATD particle-in-cell step on
 * AMD Instinct MI355X (gfx950).
 *
 * Scheme: Zoni et al., "A hybrid nodal-staggered pseudo-spectral
 * electromagnetic particle-in-cell method with finite-order centering",
 * arXiv 2106.12919.  One step follows the hybrid cycle of Sec. 2:
 * centre E,B from the Yee grid to the nodes -> gather on the nodes and push ->
 * deposit rho, J on the nodes -> centre J from the nodes to the Yee grid ->
 * standard PSATD update of E,B on the Yee grid in Fourier space (Sec. 4.2).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Normalised units: c = eps0 = mu0 = 1.  Charges and masses are in units of
 *   the elementary charge and the electron mass.
 * - Grids are triply periodic, nx*ny*nz points, stored C-order (z fastest).
 *   Node (i,j,k) sits at (i*dx, j*dy, k*dz).  A Yee component is stored at the
 *   index of the node at or below its position: E^x[i][j][k] is the value at
 *   ((i+1/2)dx, j dy, k dz), B^x[i][j][k] at (i dx, (j+1/2)dy, (k+1/2)dz), etc.
 *   (App. A list of positions; J sits with E, rho is nodal).
 * - Every array argument is caller-owned DEVICE memory on the context's
 *   device, in the context's dtype (float for PIC_F32, double for PIC_F64),
 *   aligned to at least 16 bytes.  The library keeps no pointer beyond a call.
 * - Every call enqueues work asynchronously on the context's HIP stream and
 *   returns without waiting (pic_sync waits).  Errors detected on the host are
 *   returned before anything is enqueued; asynchronous device errors surface as
 *   PIC_EHIP at a later call or at pic_sync.  pic_last_error gives the text.
 * - A context is not thread-safe: use one context per host thread/stream.
 */
#ifndef PIC_H
#define PIC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pic_ctx_s* pic_ctx;

typedef enum {
  PIC_OK = 0,
  PIC_EINVAL = 1,        /* bad argument: null pointer, out-of-range value, dtype mismatch */
  PIC_EUNSUPPORTED = 2,  /* valid but not supported (grid size, order) */
  PIC_EHIP = 3,          /* HIP runtime or kernel error */
  PIC_ENOMEM = 4,        /* device allocation failed */
  PIC_ESTATE = 5         /* call order violated (e.g. destroyed context) */
} pic_status;

typedef enum { PIC_F32 = 0, PIC_F64 = 1 } pic_dtype;

/* pic_center directions and field selectors */
enum { PIC_N2S = 0, PIC_S2N = 1 };
enum { PIC_J = 0, PIC_E = 1, PIC_B = 2 };
/* pic_deposit modes */
enum { PIC_DEP_RHO_AND_J = 0, PIC_DEP_RHO_ONLY = 1 };
/* pic_params.flags */
enum {
  /* Spectral current correction (standard PSATD only; v_gal = 0, not PIC_AVERAGED).  The direct
   * deposition of the hybrid cycle does not satisfy the discrete continuity equation, and the
   * paper leaves charge conservation to future work (Sec. 6).  With this flag the field solve
   * first projects J^{n+1/2} onto the Fourier-space continuity equation of App. A with the
   * solver's own modified wave number, in the paper's Fourier convention:
   *   J <- J - [k]_s ([k]_s . J - i (rho^{n+1} - rho^n) / dt) / |[k]_s|^2
   * (modes with |[k]_s| = 0 keep J: k = 0, whose charge the deposition conserves exactly, and
   * with PIC_NODAL_SOLVER the Nyquist planes where [k]_c vanishes).  The change is a discrete
   * gradient, so B and the transverse current are untouched; since the update carries Gauss's
   * law exactly when continuity holds, a Gauss-consistent state stays so after every step.
   * Applies to psatd_push_fields, pic_step and their reverse modes; J_stag (J_nod with the nodal
   * solver) keeps the deposited, uncorrected current. */
  PIC_CURRENT_CORRECTION = 1u << 0,
  /* Bitwise run-to-run reproducibility: every output of pic_step, pic_deposit and pic_gather_push
   * depends only on the inputs and not on the order in which the particles of a tile are visited
   * or in which the device schedules work.  The deposition accumulates in fixed point (integer
   * additions, exact in any order); with this flag each tile's fixed-point scale is chosen from
   * its particle count and largest contribution instead of a floating-point sum (at most
   * log2(particles per tile) fewer bits of headroom), and pic_step keeps every species in the
   * caller's order (as PIC_KEEP_ORDER), so particle outputs are in a fixed order too.  The
   * fully staggered cycle returns PIC_ENOMEM rather than fall back to its untiled deposition
   * (float atomics) when scratch cannot be allocated. */
  PIC_DETERMINISTIC = 1u << 1,
  /* pic_step applies the finite-order centering of J (nodes -> Yee) and of the updated
   * E, B (Yee -> nodes) as the stencils' exact Fourier symbols inside the per-mode
   * update: on the periodic grid the stencil of Sec. 3 is that multiplication (App. C),
   * so the results equal the real-space cycle up to rounding, without the two
   * real-space centering passes per step.  At return E_stag, B_stag, J_stag, rho_old and
   * the particles are as in the real-space cycle; E_nod, B_nod hold the centred fields of
   * the final time level (the real-space cycle leaves those of the last step's start).
   * pic_center and psatd_push_fields are unaffected. */
  PIC_SPECTRAL_CENTERING = 1u << 2,
  /* Nodal comparison solver (Sec. 2, the standard nodal PSATD cycle the hybrid scheme is
   * measured against): every field sits on the nodes, derivatives use the centered
   * modified wave number [k]_c (Sec. 4.1 eq. centered_modified_wave_number) with no
   * half-cell phase, and no centering is done.  The arrays named E_stag, B_stag then hold
   * the NODAL state, which pic_gather_push inside pic_step reads directly; pic_step leaves
   * E_nod, B_nod and J_stag untouched; psatd_push_fields reads J_stag as the nodal current.
   * Excludes PIC_SPECTRAL_CENTERING. */
  PIC_NODAL_SOLVER = 1u << 3,
  /* pic_step keeps every species in the caller's order: each step sorts the particles by
   * tile through a permutation (one counting sort per step) instead of regrouping the
   * arrays.  The results are those of the default cycle up to the summation order of the
   * deposition.  For callers that follow particles by index across steps (the reverse
   * mode, pic_step_adjoint). */
  PIC_KEEP_ORDER = 1u << 4,
  /* Averaged Galilean PSATD (Sec. 4.4, eqs. eq_update_B/E_with_rho_averaged): E, B advance with
   * the Galilean update (v_gal, possibly zero), and each update also writes the averaged fields
   * <E>^{n+1}, <B>^{n+1} (coefficients Psi1, Psi2, Y1..Y4 of Sec. 4.4, built in FP64) into
   * pic_fields.E_avg, B_avg on the Yee grid: the means of the step's solution, continued with
   * the same J, over [t_n + dt/2, t_n + 3 dt/2].  pic_step gathers the particles' fields from
   * E_avg, B_avg (centred to the nodes): on entry they hold the averaged fields of time n (the
   * caller sets them, e.g. to E, B at the first step).  Excludes PIC_SPECTRAL_CENTERING. */
  PIC_AVERAGED = 1u << 5,
  /* The fully staggered cycle the paper compares the hybrid one against (Sec. 2; the staggered runs
   * of Sec. 5.2-5.3): no centering; pic_gather_push interpolates every component of E_stag, B_stag
   * from its own Yee positions (the B-spline centred on x_i + delta_c), pic_deposit adds J^d onto
   * the Yee positions of J^d (into J_stag; rho^{n+1} stays nodal) and pic_step runs that cycle with
   * the same staggered PSATD update.  Particles keep the caller's order.  Tiled like the hybrid
   * gather and deposition, with six shifted stencils (a comparison path, not tuned).  Excludes PIC_NODAL_SOLVER,
   * PIC_SPECTRAL_CENTERING and PIC_AVERAGED; no reverse mode. */
  PIC_STAGGERED_CYCLE = 1u << 6
};

typedef struct {
  int32_t nx, ny, nz;     /* each even, of the form 2^a 3^b, 8 <= n <= 1024 */
  double dx, dy, dz;      /* cell sizes, > 0 */
  double dt;              /* time step, 0 < c*dt <= min(dx,dy,dz) (a particle moves < 1 cell per step) */
  int32_t shape_order;    /* particle shape: 1 = linear (CIC), 3 = cubic B-spline */
  int32_t center_order;   /* finite-order centering 2m, even, 2..32, with 2m <= min(nx,ny,nz) (Sec. 3) */
  int32_t psatd_order;    /* order 2m_p of the staggered modified wave number [k]_s, even 2..64; 0 = infinite */
  pic_dtype dtype;        /* precision of fields, particles, FFTs; tables are always built in FP64 */
  uint32_t flags;         /* an OR of the flags above (exclusions as documented with each); other bits are rejected */
  double v_gal[3];        /* Galilean velocity (in units of c), |v_gal| < 1; all zero = standard PSATD.  Nonzero:
                           * the standard Galilean PSATD update of Sec. 4.3 (eqs.
                           * eq_update_B/E_with_rho_galilean; coefficients built in FP64 from Sec. 4.1
                           * W = v_gal . [k]_c, theta = exp(i W dt/2), chi_1, X1..X4), on the grid of
                           * coordinates moving with v_gal: pic_gather_push and pic_step move particles
                           * by (v - v_gal) dt and deposit J at x^{n+1} - (v - v_gal) dt/2.  Requires a
                           * finite psatd_order and (c + |v_gal|) dt <= min(dx, dy, dz); not with
                           * PIC_SPECTRAL_CENTERING; no reverse mode. */
} pic_params;

/* One particle species, structure of arrays, caller-owned device memory.
 * Position = node index + offset: the particle lies at
 * ((i + off[0]) dx, (j + off[1]) dy, (k + off[2]) dz) with cell = (i*ny + j)*nz + k
 * and every offset in [0, 1).  u = gamma v / c.  Immobile species use m = INFINITY:
 * they are never pushed and deposit charge only. */
typedef struct {
  int64_t n;              /* number of particles (>= 0) */
  int32_t* cell;          /* [n] linear cell index */
  void* off[3];           /* [n] each, dtype */
  void* u[3];             /* [n] each, dtype */
  void* w;                /* [n] per-particle weight (dtype), or NULL to use w_const */
  double w_const;         /* weight used when w == NULL */
  double q, m;            /* charge and mass of one weight unit */
} pic_species;

/* Grid arrays of one step, each nx*ny*nz elements of dtype (see conventions). */
typedef struct {
  void* E_stag[3];        /* E on the Yee grid at time n (state) */
  void* B_stag[3];        /* B on the Yee grid at time n (state) */
  void* E_nod[3];         /* E centred to the nodes (output of pic_center S2N) */
  void* B_nod[3];         /* B centred to the nodes */
  void* J_nod[3];         /* J^{n+1/2} on the nodes (output of pic_deposit) */
  void* J_stag[3];        /* J^{n+1/2} on the Yee grid (output of pic_center N2S) */
  void* rho_old;          /* rho^n on the nodes */
  void* rho_new;          /* rho^{n+1} on the nodes */
  const void* rho_static; /* optional static background charge added by pic_deposit, or NULL */
  void* E_avg[3];         /* PIC_AVERAGED: averaged E, B on the Yee grid (see the flag); else unused, may be NULL */
  void* B_avg[3];
} pic_fields;

/* Create a context on the current HIP device.  Validates *p, builds in FP64 on
 * the host the Fornberg coefficients (Sec. 3, eq. eq_Fornberg_staggered), the
 * staggered modified wave numbers [k]_s (Sec. 4.1) and the per-mode PSATD
 * coefficients C, S/w_s, X1, X2, X3 (Sec. 4.2; X4 = -S/w_s; w_s = 0 takes the
 * limits), casts them to dtype and uploads them with the FFT plans and
 * the k-space work buffers (owned by the context).  hip_stream may be NULL
 * (null stream).  On error *out is set to NULL and the error text is available
 * from pic_last_error(NULL). */
pic_status pic_init(const pic_params* p, void* hip_stream, pic_ctx* out);

/* Free everything the context owns.  Waits for its stream first. */
pic_status pic_destroy(pic_ctx ctx);

/* Change the stream later calls enqueue on. */
pic_status pic_set_stream(pic_ctx ctx, void* hip_stream);

/* Deposit rho^{n+1} and J^{n+1/2} on the nodal grid (Sec. 2, hybrid cycle; time
 * levels of Sec. 4.2).  Called after pic_gather_push, so positions are x^{n+1}
 * and momenta u^{n+1/2}.  Zeroes f->rho_new, adds f->rho_static (if not NULL),
 * then adds sum_p q w S(x_p^{n+1} - x_i)/dV.  With PIC_DEP_RHO_AND_J it also zeroes
 * f->J_nod and adds sum_p q w v_p S(x_p^{n+1/2} - x_i)/dV with
 * x^{n+1/2} = x^{n+1} - dt v/2 (direct deposition).  S is the B-spline of
 * shape_order.  Immobile species contribute to rho only.  nsp >= 0 species. */
pic_status pic_deposit(pic_ctx ctx, const pic_species* sp, int nsp, pic_fields* f, int mode);
/* (With PIC_STAGGERED_CYCLE: J^d onto the Yee positions of J^d, into f->J_stag; see the flag.) */

/* pic_deposit for callers that cannot allocate device memory: code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc.  Same arguments, results and kernels as
 * pic_deposit (hybrid cycle), but the per-call tile sort of each species (two int32 per
 * particle), which pic_deposit keeps in context scratch allocated on a species' first use, lives
 * in a static device array of 32 MiB that the library holds on each GPU until the process ends;
 * the call itself allocates and frees nothing (pic_init, which allocates, must have run).
 * Limits and errors: at most 4,194,304 particles per species per call (PIC_EUNSUPPORTED beyond);
 * PIC_EUNSUPPORTED with PIC_STAGGERED_CYCLE; PIC_EHIP if the array's device address could not be
 * taken at pic_init.  Every call on one GPU (any context, any stream) shares that array: calls
 * that overlap in time on one GPU race and must be ordered by the caller. */
pic_status pic_deposit_noalloc(pic_ctx ctx, const pic_species* sp, int nsp, pic_fields* f, int mode);

/* Finite-order centering (Sec. 3, eq. staggered_finite_sum, order center_order):
 *   dir = PIC_N2S, what = PIC_J : J_nod -> J_stag, J^d along axis d,
 *         f_{j+1/2} = sum_n alpha^s_{m,n} (f_{j+n} + f_{j+1-n}) / 2;
 *   dir = PIC_S2N, what = PIC_E : E_stag -> E_nod, E^d along axis d,
 *   dir = PIC_S2N, what = PIC_B : B_stag -> B_nod, B^d along the two other axes,
 *         f_j = sum_n alpha^s_{m,n} (f_{j+n-1/2} + f_{j-n+1/2}) / 2.
 * The two directions are exact transposes of each other, so the remaining pairs give the
 * adjoints (reverse mode) of the three above:
 *   (PIC_S2N, PIC_J): J_stag -> J_nod, (PIC_N2S, PIC_E): E_nod -> E_stag,
 *   (PIC_N2S, PIC_B): B_nod -> B_stag (the same two axes).
 * Other values of dir or what return PIC_EINVAL. */
pic_status pic_center(pic_ctx ctx, int dir, int what, pic_fields* f);

/* Standard PSATD update on the staggered grid (Sec. 4.2, eqs.
 * eq_update_B_with_rho_standard and eq_update_E_with_rho_standard) in the
 * Fourier convention of App. A (each component transformed at its own Yee
 * position).  Reads E_stag, B_stag (time n), J_stag, rho_old, rho_new and
 * overwrites E_stag, B_stag with time n+1.  Uses 11 forward and 6 inverse
 * real 3D FFTs. */
pic_status psatd_push_fields(pic_ctx ctx, pic_fields* f);

/* Reverse mode of psatd_push_fields (the adjoint of a linear map, for differentiating a
 * loss through the field solve): on entry E_stag, B_stag hold dL/dE^{n+1}, dL/dB^{n+1};
 * on return E_stag, B_stag hold dL/dE^n, dL/dB^n and J_stag, rho_old, rho_new hold
 * dL/dJ^{n+1/2}, dL/drho^n, dL/drho^{n+1} (overwritten).  Per mode it applies the
 * conjugate transpose of the update of Sec. 4.2 (for a time-symmetric vacuum update this
 * is the time-reversed update, App. B); the transforms pair as FFT^H = N IFFT.  Honours
 * PIC_NODAL_SOLVER. */
pic_status psatd_push_fields_adjoint(pic_ctx ctx, pic_fields* f);

/* Gather E_nod, B_nod at x^n with the shape_order B-spline (one weight set for
 * all six nodal components) and advance every mobile species with the
 * relativistic Boris scheme: u^{n-1/2} -> u^{n+1/2}, x^{n+1} = x^n + dt u/gamma,
 * periodic wrap of cell and offset. */
pic_status pic_gather_push(pic_ctx ctx, const pic_fields* f, pic_species* sp, int nsp);
/* (With PIC_STAGGERED_CYCLE: from E_stag, B_stag, each component at its own Yee positions.) */

/* nsteps >= 0 complete hybrid cycles.  State on entry: E_stag, B_stag at time n,
 * particles at x^n with u^{n-1/2}, rho_old = rho^n.  Each step runs
 * S2N centering -> gather+push -> deposit -> N2S centering -> PSATD update.  (When every
 * axis length is one of 64, 128, 256, 384, 768, the steps of a call before its last apply
 * both centerings inside the transforms, to whole lines of the centred axis, with the same
 * stencil: the results equal those of the separate passes up to rounding.)  On
 * return E_stag, B_stag, particles and rho_old are at time n+nsteps, and E_nod,
 * B_nod, J_nod, J_stag, rho_new hold the intermediates of the last step.  E and
 * B stay in Fourier space between the steps of one call (7 forward transforms on
 * entry, then 4 forward and 6 inverse per step).  Particles of each species may
 * be reordered (all per-particle arrays together) to group them by grid tile, unless
 * PIC_KEEP_ORDER (or PIC_STAGGERED_CYCLE).  The flags of pic_init select the variants:
 * PIC_SPECTRAL_CENTERING, PIC_NODAL_SOLVER, PIC_STAGGERED_CYCLE, v_gal (Galilean) and
 * PIC_AVERAGED (the particles then see E_avg, B_avg), as documented with each flag. */
pic_status pic_step(pic_ctx ctx, pic_fields* f, pic_species* sp, int nsp, int nsteps);

/* Adjoints of one species' particle state (caller-owned device arrays of dtype, n each). */
typedef struct {
  void* off[3];           /* dL/d offset (per cell of the axis: the derivative w.r.t. the position in cells) */
  void* u[3];             /* dL/du */
} pic_species_adjoint;

/* Reverse mode of one step of pic_step (Sec. 2 cycle), for differentiating a loss through
 * the cycle: given the state at time n and the adjoint of the state at n+1, returns the
 * adjoint of the state at n.  The stages are taken in reverse order: the conjugate-
 * transposed field solve (as psatd_push_fields_adjoint), the transposed centerings
 * (pic_center's transposed pairs), and per particle the adjoints of the deposition, the
 * move, the relativistic Boris push and the gather (the B-spline and its derivative), whose
 * field adjoints are spread back onto the nodes with the particle's shape (the transpose of
 * the gather).  Forward quantities of the step are recomputed from the state at n.
 *   f:   the state at n, as pic_step reads it: E_stag, B_stag (read; PIC_NODAL_SOLVER: the
 *        nodal state); E_nod, B_nod are workspace (overwritten; unused with the nodal solver).
 *   sp:  the nsp species at time n (x^n, u^{n-1/2}), in the order in which asp indexes them
 *        (pic_step with PIC_KEEP_ORDER leaves that order unchanged); read only.
 *   adj: in:  E_stag, B_stag = dL/dE^{n+1}, dL/dB^{n+1}; rho_new = dL/drho^{n+1} (the
 *             adjoint of the next step's rho_old);
 *        out: E_stag, B_stag = dL/dE^n, dL/dB^n; rho_old = dL/drho^n;
 *        J_nod, J_stag, E_nod, B_nod and rho_new are workspace (overwritten).
 *   asp: per species, in dL/dx^{n+1}, dL/du^{n+1/2}; out dL/dx^n, dL/du^{n-1/2} (in place).
 * rho_static is constant (no adjoint).  Immobile species receive position adjoints from
 * the charge they deposit.  Every array must be distinct from the others.  The adjoint of
 * the spectral-centering cycle is that of the real-space cycle (the same map). */
pic_status pic_step_adjoint(pic_ctx ctx, pic_fields* f, const pic_species* sp, int nsp, pic_fields* adj,
                            const pic_species_adjoint* asp);

/* Wait for the context's stream; returns PIC_EHIP if a device error occurred, and
 * PIC_EINVAL if particles with a cell index outside [0, nx*ny*nz) were skipped by
 * pic_gather_push / pic_deposit / pic_step since the last pic_sync (the kernels
 * never access memory through such an index). */
pic_status pic_sync(pic_ctx ctx);

/* Diagnostics, computed on the device and accumulated in FP64 (synchronous):
 * out[0] = field energy W = 1/2 sum (|E|^2 + |B|^2) dV of the Yee-grid state
 * (Sec. 2 item iii), out[1] = total charge sum(rho_old) dV. */
pic_status pic_diagnostics(pic_ctx ctx, const pic_fields* f, double out[2]);

/* Gauss's-law residual of the state (synchronous; FP64 accumulation): *out =
 * || [k]_s . E_hat + i rho_hat / eps0 || / || rho_hat / eps0 || over all modes, in the paper's Fourier
 * convention (App. A; Gauss's law is the constraint the PSATD update of Sec. 4.2 preserves), from
 * E_stag and rho_old (|| . || alone when rho is zero).  With PIC_NODAL_SOLVER, [k]_c and the nodal
 * E.  Uses the context's k-space scratch (not during another call on the same context). */
pic_status pic_gauss_residual(pic_ctx ctx, const pic_fields* f, double* out);

/* Continuity residual of a step's sources (synchronous; FP64 accumulation): *out =
 * || (rho_hat^{n+1} - rho_hat^n) / dt + i [k]_s . J_hat || / || (rho_hat^{n+1} - rho_hat^n) / dt ||
 * over all modes, in the paper's Fourier convention (App. A), from rho_old = rho^n, rho_new =
 * rho^{n+1} and J_stag = J^{n+1/2} on the Yee grid (with PIC_NODAL_SOLVER: [k]_c and J_nod).  The
 * direct deposition of Sec. 2 does not conserve charge, so this is a reported quantity, not zero;
 * the field solve of Sec. 4.2 keeps Gauss's law exactly when it is zero.  (|| . || alone when rho
 * does not change.)  Uses the context's k-space scratch (not during another call on the context). */
pic_status pic_continuity_residual(pic_ctx ctx, const pic_fields* f, double* out);

/* Per-stage timing with HIP events on the context stream.  When enabled, each
 * stage launch of pic_step is bracketed by events; pic_stage_times returns, for
 * stage s < nstage, the accumulated milliseconds and the number of launches since
 * the last reset.  Stage names: pic_stage_name(s). */
pic_status pic_profile(pic_ctx ctx, int enable);
pic_status pic_stage_times(pic_ctx ctx, double* ms, int64_t* count, int nstage);
const char* pic_stage_name(int s);
int pic_num_stages(void);

/* ---- Closed-form diagnostics of the discrete scheme: host functions in FP64, no context
 * and no GPU needed.  Every output is a caller-owned HOST array.  On a bad argument they
 * return PIC_EINVAL (text in pic_last_error(NULL)). */

/* Modified wave numbers of an axis of n points and spacing d at finite-difference order
 * `order` (even, 0..64; 0 = the exact k): out[i] for the DFT index i, whose signed
 * frequency is f = i, or i - n for i > (n-1)/2 (even n: index n/2 is -n/2), k = 2 pi f/(n d).
 * kind 0: staggered [k]_s (Sec. 4.1 eq. staggered_modified_wave_number, coefficients
 * eq. eq_Fornberg_staggered); kind 1: centered [k]_c (eq. centered_modified_wave_number,
 * eq. eq_Fornberg_centered).  The standard PSATD solver propagates vacuum waves at
 * w = c |[k]| exactly (App. B eq. vacuum_disprel_psatd), so out[i] / k is the numerical
 * phase velocity over c along the axis (Sec. 2, dispersion figure): n doubles. */
pic_status pic_modified_wavenumber(int32_t n, double d, int32_t order, int32_t kind, double* out);

/* Fourier factor of the finite-order centering of order center_order = 2m (even, 2..64)
 * along an axis of n points (App. C): zeta(k) = sum_n alpha^s_{m,n} cos(k (n - 1/2) d), at
 * the DFT indices as above (k d = 2 pi f / n, so d drops out).  Its deviation from 1 is what
 * governs the mitigation of the numerical Cherenkov instability (App. C): n doubles. */
pic_status pic_centering_factor(int32_t n, int32_t center_order, double* out);

/* Stencil extent (Sec. 2 item (ii), eq. eq_stencil_extent) along `axis` (0, 1, 2) of one
 * standard PSATD coefficient, coefficient 0 = C, 1 = S/w, 2 = X1, 3 = X2, 4 = X3, for the
 * grid, cell sizes, dt and psatd_order of *p, with [k]_s, or [k]_c when p->flags has
 * PIC_NODAL_SOLVER:  Gamma(x_j) = | (1/(N_b N_c)) sum_{k_b, k_c} [F^-1_axis g](x_j, k_b, k_c) |
 * for j = 0 .. n_axis - 1 (cells from the origin; j > n/2 is the distance n - j on the
 * other side): n_axis doubles.  Costs one coefficient evaluation per mode of the grid. */
pic_status pic_stencil_extent(const pic_params* p, int32_t axis, int32_t coefficient, double* out);

/* ---- Measurement support (no context). */

/* Throughput of integer LDS atomics on the current device, the bound of the fixed-point
 * deposition: every workgroup issues `iters` (a multiple of 16, 16 .. 2^20) adds per thread of
 * width_bits (32: ds_add_u32 with the 32 lanes of each half wave on distinct words modulo 32;
 * 64: ds_add_u64 with the 16 lanes of each quarter wave on distinct words modulo 16, the patterns
 * of the deposition's dealt order) into its own LDS array; *lane_ops_per_s_per_cu receives the
 * lane operations per second per compute unit.  Synchronous, on the null stream; allocates a few
 * bytes of device memory.  PIC_EINVAL for bad arguments, PIC_EHIP if a HIP call fails. */
pic_status pic_probe_lds_atomics(int width_bits, int iters, double* lane_ops_per_s_per_cu);

/* Text of the last error of ctx (or of the last failed pic_init when ctx is NULL). */
const char* pic_last_error(pic_ctx ctx);
const char* pic_strerror(pic_status s);

#ifdef __cplusplus
}
#endif

#endif /* PIC_H */
