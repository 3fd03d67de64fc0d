/*
 * tpl.h -- C ABI of the MI355X implementation of the two-fluid kinetic scheme
 * for dilute polymer solutions of Singh, Subramanian & Ansumali,
 * "Two-fluid kinetic theory for dilute polymer solutions" (arXiv:2201.10132).
 *
 * One time step advances two populations on one 2-D periodic lattice:
 *   - solvent: D2Q9 populations (Sec. VI.A);
 *   - polymer: D4Q25 populations over (r, Q) (Sec. VI.B, Table I), i.e. at
 *     every r-node a disk of Q-nodes (|Q| < NQ/2, bounce-back on the circle,
 *     Sec. VI.C) with 25 populations each;
 * coupled through the mixture velocity and the dumbbell spring term
 * (imposed fluxes of Sec. V), relaxed by the component-momentum
 * quasi-equilibrium model (Sec. IV-V) with the trapezoidal time
 * discretisation made explicit (Sec. VI.C), and driven by the Kolmogorov
 * body force of Sec. VII.
 *
 * Conventions
 *   - Lattice units dx = dt = dQ = 1, c_s^2 = 1/3.
 *   - Every call returns 0 (TPL_OK) or a negative TPL_E* code; no C++
 *     exception crosses this boundary.  tpl_last_error() returns a
 *     thread-local message describing the last failure of the calling thread.
 *   - A context is used by one host thread at a time.
 *   - Host buffers passed in are owned by the caller and only read/written
 *     during the call.  Device buffers are owned by the context (or by the
 *     caller after tpl_adopt_buffers).
 *   - Canonical array layouts (row index y, column index x, r = y*nx + x):
 *       solvent populations  XS[9][ny][nx]
 *       polymer populations  XP[25][nqd][ny][nx]
 *       polymer density      psi[nqd][ny][nx]      (psi = sum_k XP_k)
 *       mixture velocity     U[2][ny][nx]
 *     D2Q9 order: (0,0) (1,0) (0,1) (-1,0) (0,-1) (1,1) (-1,1) (-1,-1) (1,-1).
 *     D4Q25 order: k = 0 rest; k = 1 + 4p + s for coordinate pairs
 *     p = (vx,vy) (vx,Qx) (vx,Qy) (vy,Qx) (vy,Qy) (Qx,Qy) and sign pairs
 *     s = (+,+) (+,-) (-,+) (-,-).  Q-disk nodes Q = (a + 1/2 - NQ/2,
 *     b + 1/2 - NQ/2) with |Q| < NQ/2, numbered row by row (b outer).
 */
#ifndef TPL_H
#define TPL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  TPL_OK = 0,
  TPL_EINVAL = -1,    /* invalid argument or parameter combination */
  TPL_ENOMEM = -2,    /* device or host allocation failed */
  TPL_EHIP = -3,      /* a HIP runtime call failed */
  TPL_ESTATE = -4,    /* call not allowed in the context's current state */
  TPL_EUNSTABLE = -5, /* the state holds NaN/Inf: the run diverged */
  TPL_EREJECTED = -6  /* a learned correction was rejected by its drift gate */
};

/* Storage forms of the populations (arithmetic is FP64 in all of them):
 *   TPL_FP64     FP64 values
 *   TPL_FP32     FP32 deviations from an x-invariant FP32 reference (the
 *                base state), FP64 per-node fields
 *   TPL_BF16     solvent and psi as TPL_FP32; the polymer populations as the
 *                BF16 rounding (nearest even, 8 significant bits) of their
 *                deviation from the same reference, except the rest
 *                population (it never leaves its node), kept in FP32 and
 *                carrying the rounding residual of the other 24, so that the
 *                stored density of every (r, Q)-node, and the mass, are exact
 *                to FP32 (56 bytes per (r, Q)-node against 104 for FP32 and
 *                208 for FP64).  Its error is set by
 *                the size of the deviations: small near the reference (a
 *                perturbed, converged base state), large where the state has
 *                moved far from it (a base state still spinning up)
 */
enum { TPL_FP64 = 0, TPL_FP32 = 1, TPL_BF16 = 2 };
enum { TPL_SOLVENT = 0, TPL_POLYMER = 1 };

#define TPL_NFIELDS 10
#define TPL_NDIAG 9

typedef struct tpl_ctx tpl_ctx;

/* Kolmogorov forcing (Sec. VII): body force F0 sin(2 pi periods y / ny) on the
 * solvent, F0 = nu u0 k^2 (F = eta U / l^2 with rho = 1). */
typedef struct {
  int periods;
  double u0; /* lattice velocity scale, <= 0.1 */
} tpl_forcing;

typedef struct {
  double step;      /* completed time steps since tpl_init */
  double mass_S;    /* sum of solvent populations */
  double mass_P;    /* sum of polymer populations */
  double mom_x;     /* sum of population momenta, both species */
  double mom_y;
  double amplitude; /* tpl_perturbation_amplitude() */
  double enstrophy; /* (1/2) sum omega^2, omega = dUy/dx - dUx/dy (central) */
  double qrms;      /* sqrt(sum psi |Q|^2 / sum psi) / (NQ/2) */
  double min_psi;   /* smallest psi over all (r, Q) nodes */
} tpl_diag;

/* Create a context for an nx x ny periodic lattice (nx = 1 is the x-invariant
 * column).  Parameters (Sec. VII): Re = u0 l / nu with l = ny / (2 pi periods)
 * and nu the solution viscosity; beta = eta_s / (eta_s + eta_p);
 * Wi = u0 lambda / l (Wi = 0: Newtonian limit, no elastic stress).  Derives
 * every lattice parameter and builds the Q-disk tables on the host; no device
 * memory is touched until tpl_init.  Returns NULL on error (tpl_last_error):
 * nx < 1, ny < 4 periods, nx ny >= 2^29, Re <= 0, Wi < 0, beta outside (0, 1], u0 outside
 * (0, 0.1], or tau1 > tau2 for either species (H-theorem ordering, Sec. IV). */
tpl_ctx *tpl_create(int nx, int ny, double Re, double Wi, double beta,
                    tpl_forcing forcing);

/* Set a parameter before tpl_init (TPL_ESTATE afterwards, except for the
 * launch/timing knobs qsplit, group_x, group_y, group_sync, autotune and
 * time_kernels and the health-check knobs diag_every, psi_floor and
 * keep_good, which may be set at any time and change no result;
 * TPL_EINVAL for an unknown key or a value out of range).  Keys and defaults:
 *   nq 16         Q points per axis (even, 4..48)
 *   spring 0      0 = FENE (Warner), 1 = Hookean
 *   b 25          FENE extensibility; sigma = (nq/2) / sqrt(b)
 *   phi 0.01      polymer mass fraction
 *   tau_drag 0    solvent drag time (model 1: tau2_S, model 2: tau1_S);
 *                 0 = automatic: 1 (model 1) or tau2_S (model 2)
 *   tau_ratio_p 1 polymer tau1 / tau2
 *   force_scale 1 multiplies F0
 *   lambda 0      > 0: polymer relaxation time in steps instead of Wi l / u0
 *   drift_cap 0.2 cap on the Q-drift D_Q |F/kT| per step (0 = none); it
 *                 keeps the linear Q-space equilibrium positive near the
 *                 FENE singularity, which needs a drift below c_s^2 = 1/3
 *                 per step less the flow term K Q; 0.2 leaves that room.
 *                 A tighter cap binds inside the bulk of the FENE rest
 *                 distribution where tau2_P is large (0.1 stretches it by
 *                 18 % at tau2_P = 0.54)
 *   drift_relax 1 also cap that drift at drift_relax (2 - omega_P), the
 *                 damping rate of the polymer's non-conserved moments,
 *                 omega_P = 2 / (2 tau1_P + 1) (0 = none)
 *   qe_model 1    quasi-equilibrium model (Sec. V): 1 = component momenta
 *                 quasi-conserved (viscosity c_s^2 tau1_S, drag time
 *                 tau2_S = tau_drag, D_Q = c_s^2 tau2_P); 2 = component
 *                 stresses quasi-conserved (viscosity c_s^2 tau2_S, drag time
 *                 tau1_S = tau_drag <= tau2_S, D_Q = c_s^2 tau1_P,
 *                 tau2_P = tau1_P / tau_ratio_p); in a batch every
 *                 instance takes the same model, model (ii) with
 *                 spring_shift 0
 *   precision 0   TPL_FP64, TPL_FP32 or TPL_BF16 population storage
 *   inplace 0     1 = one population array instead of two, streamed in place
 *                 (Sec. VI streaming and Q-disk bounce-back, by the AA
 *                 pattern of Bailey et al., ICPP 2009): steps alternate
 *                 between pulling from the neighbours and writing back into
 *                 the locations read, and reading and writing the node's
 *                 own locations; results are bitwise those of the
 *                 two-array step.  Halves the population memory.  FP64 and
 *                 FP32 only, nx a multiple of 64, one Q-slice (qsplit is
 *                 ignored); a batch sets it for all its instances
 *                 (tpl_batch_set_param).  After an odd number of steps
 *                 the populations are held in streamed order: the calls
 *                 that read or write populations (tpl_get_state with XS or
 *                 XP, tpl_set_state, tpl_get_window, tpl_get_populations,
 *                 tpl_set_populations, tpl_save, tpl_restrict) return
 *                 TPL_ESTATE until one more step is taken; observables,
 *                 diagnostics and the amplitude are available after every
 *                 step.  The autotuner times its shapes on the first
 *                 tpl_step of at least 24 steps, as real steps
 *   gradients 0   time level of the velocity gradient and of the spring
 *                 term's psi gradient (the paper leaves it open): 0 = the
 *                 previous step's observables (one pass); 1 = this step's,
 *                 formed from the pulled populations before the step (three
 *                 more launches, about 1.5x the bytes; FP64 and FP32 forms;
 *                 a batch sets it for all instances)
 *   spring_shift 0  form of the spring term of the imposed polymer flux
 *                 (Sec. V, the force times psi at the two beads): 0 = its
 *                 first-order Taylor form kappa Fhat (Q . grad psi); 1 = the
 *                 shift itself, kappa Fhat [psi(r + Q/2) - psi(r - Q/2)] with
 *                 psi between nodes by periodic bilinear interpolation (one
 *                 more launch sums it over Q); FP64 and FP32 forms, in place
 *                 or not; with gradients 1 the sum is taken over this step's
 *                 psi and replaces the M pass; a batch sets it for all
 *                 instances
 *   pert_modes 1  0 = single x-mode, 1 = multimode perturbation
 *   init_mode 0   base state: 0 = the forced x-invariant state reached by a
 *                 pre-run of the scheme on one column (pre_steps); 1 = the
 *                 closed-form laminar state of Hookean dumbbells (Oldroyd-B
 *                 profile with the populations' stress diffusion, both
 *                 species at their equilibria; Sec. VII forcing, Sec. V
 *                 fluxes), for spring 1, qe_model 1 and Wi > 0 (TPL_EINVAL
 *                 from tpl_init otherwise; batches take 0 only)
 *   pre_steps -1  base-state column steps (-1 = 5 max(l^2/nu, lambda))
 *   qsplit 0      Q-slices per r-tile in the step kernel: 0 (automatic),
 *                 1, 2, 4 or 8 (other values round down)
 *   group_x 1, group_y 1, group_sync 0
 *                 tile groups of the step kernel: group_x x group_y tiles of
 *                 64 nodes (group_y consecutive rows) per workgroup, one wave
 *                 each, group_sync 1 = a barrier per Q-node keeps them
 *                 together; product at most 8; used with one Q-slice and
 *                 nx a multiple of 64 group_x, ny of group_y (else ignored);
 *                 a product > 1 overrides the autotuner
 *   autotune 1    1 = on the first tpl_step, time the tile-group shapes of
 *                 the full lattice (a few idempotent launches; tune_ms) and
 *                 keep the fastest; every shape gives bitwise the same step
 *   time_kernels 0  1 = time every step-kernel launch with HIP events
 *   diag_every 0  tpl_step checks the state's health every diag_every steps
 *                 (0: once, after its last step) and stops at the first
 *                 failed check (see tpl_step)
 *   psi_floor 1   tolerance of that check on the polymer density: the state
 *                 fails if min psi < -psi_floor max psi over all (r, Q)-nodes.
 *                 The linear Q-space equilibrium does not keep psi positive:
 *                 in healthy runs the outermost Q-nodes hold psi down to
 *                 about -1e-2 max psi (the 64^2 workload) and, with strongly
 *                 stretched FENE dumbbells (Wi 5 on a 16-point Q-grid),
 *                 -0.3 max psi; a diverging run goes far below
 *   keep_good 0   1 = a failed check puts back the state of the last passed
 *                 check (see tpl_step); costs a device copy of the state
 *                 (bytes_state / 2, allocated on the first such tpl_step)
 *                 and one device-to-device copy of it per check
 * Any parameter also fixes the derived values read by tpl_query. */
int tpl_set_param(tpl_ctx *ctx, const char *key, double value);

/* Read a parameter, a derived value or a size.  Keys: every tpl_set_param key
 * and nx ny nqd Re Wi beta u0 periods kf l nu nuS G tau1S tau2S tau1P tau2P
 * lambda_eff sigma R DQ F0 kappa meq Sc rhoS0 rhoP0 step bytes_XS bytes_XP
 * bytes_PSI bytes_FLD bytes_MOM bytes_state bytes_per_step
 * kernel_ms kernel_launches qsplit_used group_x_used group_y_used
 * group_sync_used tune_ms (the shape of the last tpl_step's launches)
 * inplace_odd (1: in-place populations held in streamed order).  Host only;
 * TPL_EINVAL for an unknown key. */
int tpl_query(const tpl_ctx *ctx, const char *key, double *out);

/* Bind a hipStream_t (NULL = the null stream).  All device work of the
 * context is enqueued on it. */
int tpl_set_stream(tpl_ctx *ctx, void *hip_stream);

/* Use caller-owned device memory for the state instead of allocating it.
 * Call before tpl_init.  dptrs[i] must be a device pointer of at least
 * bytes[i] bytes, 256-byte aligned, for i = 0..3 in the order returned by
 * tpl_query keys bytes_XS, bytes_XP, bytes_PSI, bytes_FLD (each holds the
 * double-buffered array; XS and XP hold one array with inplace 1).  The
 * caller keeps ownership. */
int tpl_adopt_buffers(tpl_ctx *ctx, void *const *dptrs, const size_t *bytes,
                      int n);

/* Allocate the state (TPL_ENOMEM if it does not fit), set the rest state,
 * run the forced x-invariant base state on a one-column lattice, copy it to
 * every column and add a seeded perturbation of RMS amplitude
 * perturbation * u0 (single mode: du_y = perturbation u0 sin(2 pi x/nx + phi0)).
 * Random numbers: SplitMix64 (Steele, Lea & Flood 2014) seeded by seed.
 * Synchronises before returning.  May be called again to restart. */
int tpl_init(tpl_ctx *ctx, uint64_t seed, double perturbation);

/* Advance n >= 0 time steps.  Enqueued on the bound stream; synchronises
 * before returning.  After every diag_every steps (after the last step if
 * diag_every is 0) a health check reads the mixture velocity and psi of
 * every (r, Q)-node: if any is NaN or Inf, or min psi < -psi_floor max psi
 * (psi is a density of dumbbell configurations, Sec. VI.B), the call returns
 * TPL_EUNSTABLE at once, with the cause in tpl_last_error.  With keep_good 0
 * the state and the step counter (tpl_query key step) are those of the
 * failed check; with keep_good 1 they are put back to the last check that
 * passed in this call, or to the call's start if none did (the message
 * names that step).  TPL_ENOMEM if keep_good cannot allocate its copy. */
int tpl_step(tpl_ctx *ctx, int64_t n);

/* Observables of the last completed step (step 0 = the initial state), SoA
 * [TPL_NFIELDS][ny][nx] doubles: rho, Ux, Uy, rho_P, Cxx, Cxy, Cyy, tau_xx,
 * tau_xy, tau_yy with C = sum psi Q Q^T / (sigma^2 sum psi) and
 * tau = G (M / (rho_P0 m_eq) - I), M = sum psi Q F^T / kT.  len counts
 * doubles; TPL_EINVAL if len < TPL_NFIELDS nx ny. */
int tpl_moments(tpl_ctx *ctx, double *out, size_t len);
/* Same into a device buffer of at least len doubles (no synchronisation). */
int tpl_moments_device(tpl_ctx *ctx, void *dptr, size_t len);

/* A(n) = sqrt(mean over the lattice of |U - <U>_x(y)|^2) / u0, reduced in
 * FP64 on the device.  NaN on error. */
double tpl_perturbation_amplitude(tpl_ctx *ctx);

/* FP64 totals and extremes of the current state (see tpl_diag). */
int tpl_diagnostics(tpl_ctx *ctx, tpl_diag *out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the values
 * of tpl_diagnostics, computed by the same kernels in a static working array
 * of the library (one per GPU, held until the process ends, about 0.6 MB)
 * instead of the context's lazily allocated buffer.  Calls no hipMalloc or
 * hipFree.  The calling thread's current device must be the context's.
 * TPL_EINVAL for a lattice of more than 65536 rows or the TPL_BF16 form
 * (which decodes into a buffer of its own).  Every call on a GPU shares that
 * GPU's array: calls that overlap in time on one GPU (other threads, other
 * streams) race and must be serialised by the caller. */
int tpl_diagnostics_noalloc(tpl_ctx *ctx, tpl_diag *out);

/* Whole-lattice state exchange in the canonical layouts, as doubles.  Any
 * pointer may be NULL (that array is skipped).  tpl_set_state requires a
 * context after tpl_init; it replaces populations, the lagged psi and U and
 * recomputes every derived per-node field from them. */
int tpl_get_state(tpl_ctx *ctx, double *XS, double *XP, double *psi,
                  double *U);
int tpl_set_state(tpl_ctx *ctx, const double *XS, const double *XP,
                  const double *psi, const double *U);
/* A w x h window with periodic wrap starting at (x0, y0), canonical layouts
 * with nx, ny replaced by w, h. */
int tpl_get_window(tpl_ctx *ctx, int x0, int y0, int w, int h, double *XS,
                   double *XP, double *psi, double *U);
/* One species' populations (TPL_SOLVENT or TPL_POLYMER) as doubles;
 * bytes must equal the array size. */
int tpl_get_populations(tpl_ctx *ctx, int species, void *host, size_t bytes);
int tpl_set_populations(tpl_ctx *ctx, int species, const void *host,
                        size_t bytes);

/* Checkpoint: parameters, step counter and the full state in storage
 * precision.  tpl_load requires a context created with the same lattice
 * size and parameters (the launch, timing and health knobs may differ) and
 * resumes bitwise. */
int tpl_save(tpl_ctx *ctx, const char *path);
int tpl_load(tpl_ctx *ctx, const char *path);

/* Release everything the context owns.  NULL is ignored. */
void tpl_destroy(tpl_ctx *ctx);

/* ------------------------------------------------------------------------
 * Batched form: many independent Kolmogorov lattices (instances) with their
 * own sizes and parameters, advanced together.  Every step is one launch of
 * the step kernel over the flat list of all instances' 64-node tiles; the
 * launches of graph_steps consecutive steps are replayed from one HIP graph.
 * Each instance computes exactly what a context of its own computes (same
 * kernel arithmetic, bitwise the same results); only the launch differs.
 */
typedef struct tpl_batch tpl_batch;

typedef struct {
  int nx, ny;        /* lattice */
  int periods;       /* forcing periods over ny */
  double Re, Wi, beta, u0;
  uint64_t seed;       /* perturbation seed (SplitMix64) */
  double perturbation; /* RMS amplitude / u0 of the multimode perturbation */
} tpl_instance;

/* Create n >= 1 instances, each validated as by tpl_create (NULL and
 * tpl_last_error naming the instance on failure), all stored in precision
 * (TPL_FP64 or TPL_FP32).  All work of the batch is enqueued on one HIP
 * stream: the caller's (tpl_batch_set_stream) or one the batch creates at
 * tpl_batch_init (non-blocking, default priority).  The array is copied. */
tpl_batch *tpl_batch_create(const tpl_instance *inst, int n, int precision);

/* Launch keys, settable at any time (a change after tpl_batch_init re-chooses
 * the launch shape):
 *   qsplit 0       Q-slices per tile (0: chosen by the autotuner)
 *   grid 0         workgroups per launch (0: chosen by the autotuner)
 *   group 0        consecutive tiles per workgroup, one wave each, with one
 *                  Q-slice: 1, 2, 4 or 8 (0: chosen by the autotuner)
 *   autotune 1     time the candidate shapes at tpl_batch_init (qsplit 1, 2,
 *                  4, 8 at one tile per workgroup, then groups of 2, 4, 8
 *                  tiles, then a persistent grid of one or two workgroups
 *                  per CU slot for the best) and keep the fastest; every
 *                  shape gives bitwise the same step; 0: heuristic shape
 *   graph_steps 20 steps captured per HIP graph (< 2: plain launches)
 *   time_kernels 0 1 = time tpl_batch_step with HIP events (kernel_ms)
 * Any other key is a tpl_set_param key applied to every instance before
 * tpl_batch_init (TPL_ESTATE afterwards; precision is rejected).
 * spring_shift 1 takes the shifted spring term for every instance (a
 * batched launch forms its Q-sums before each step); gradients 1 takes
 * same-step gradients for every instance (three batched launches form this
 * step's psi, M and U before each step).  These and inplace are set for the
 * whole batch: a value an instance refuses leaves every instance as it was
 * (the error returned), and tpl_batch_init returns TPL_EINVAL if an
 * instance's own setting differs from the batch's.  inplace 1
 * streams every instance in place
 * (each nx a multiple of 64; set here, not per instance): one Q-slice,
 * groups of `group` tiles (4 unless set), the shape not timed (an in-place
 * launch advances the state); graphs are captured per step-count parity;
 * an instance stepped on its own blocks tpl_batch_step (TPL_ESTATE) until
 * it is back at the batch's step parity. */
int tpl_batch_set_param(tpl_batch *b, const char *key, double value);

/* Keys: the launch keys above and instances, active (not flagged unstable),
 * unstable, items (tiles per launch), nodes (r-nodes of the active
 * instances), bytes_per_step (algorithmic bytes of the active instances),
 * bytes_state (all instances), qsplit_used, group_used, grid_used, rowtile, kernel_ms
 * (mean time of one step, needs time_kernels), kernel_steps, tune_ms, step. */
int tpl_batch_query(const tpl_batch *b, const char *key, double *out);

/* Bind a caller's hipStream_t to the batch and every instance (NULL: the
 * batch's own stream).  Discards the captured graph.  A graph is captured
 * only on a stream other than the null stream. */
int tpl_batch_set_stream(tpl_batch *b, void *hip_stream);

/* Allocate and initialise every instance as tpl_init does (base state from
 * its own column pre-run, all columns stepped together; then its seeded
 * perturbation), then choose the launch shape.  TPL_ENOMEM if the instances
 * do not fit (tpl_query key bytes_state of the instances, summed, plus about
 * 12 bytes per node of working memory).  Synchronises before returning. */
int tpl_batch_init(tpl_batch *b);

/* Advance every active instance n >= 0 steps, then check each as tpl_step
 * does (NaN/Inf, psi below -psi_floor max psi of that instance): an instance
 * that fails is flagged (tpl_batch_status), dropped from later launches and
 * keeps its last state; the others go on.  Returns TPL_OK unless a call
 * fails.  Synchronises before returning. */
int tpl_batch_step(tpl_batch *b, int64_t n);

/* tpl_perturbation_amplitude of every instance (NaN for an unstable one);
 * out holds n >= instances doubles. */
int tpl_batch_amplitudes(tpl_batch *b, double *out, int n);

/* 1 for each instance flagged unstable, else 0; n >= instances ints. */
int tpl_batch_status(const tpl_batch *b, int *unstable, int n);

/* The context of instance i, owned by the batch (do not destroy it).  Every
 * single-context call works on it (state exchange, diagnostics, checkpoint,
 * even tpl_step: the next tpl_batch_step continues from its current state). */
tpl_ctx *tpl_batch_instance(tpl_batch *b, int i);

/* Release the batch and all its instances.  NULL is ignored. */
void tpl_batch_destroy(tpl_batch *b);

/* ------------------------------------------------------------------------
 * Learned coarse-lattice correction.  A coarse lattice (the scheme above on
 * an m-times coarser grid, same Re, Wi, beta: acoustic scaling) is corrected
 * every step by a per-node network that sees the 3x3 neighbourhood of
 * (rho, Ux, Uy, Cxx, Cxy, Cyy) (54 features) and predicts the correction
 * (dJx, dJy, dtau_xx, dtau_xy, dtau_yy) of momentum and polymer stress that
 * one coarse step misses against the restricted fine solution.  The
 * correction acts as an extra body force F = dJ + div_h(dtau) (central
 * differences) in the next step.  Network: in -> 64 -> 64 -> out, exact GELU,
 * BF16 weights and activations, FP32 accumulation on the matrix cores, FP32
 * master parameters, Adam, loss = mean of squared errors of standardised
 * outputs.  Flat parameter layout (FP32): W1 [64][in], b1 [64], W2 [64][64],
 * b2 [64], W3 [out][64], b3 [out], each W acting as z = W x + b.
 */
typedef struct tpl_mlp tpl_mlp;

/* hidden must be 64, 1 <= in <= 64, 1 <= out <= 16 (else NULL, TPL_EINVAL).
 * Weights ~ U(-1/sqrt(fan_in), 1/sqrt(fan_in)) from SplitMix64(seed), zero
 * biases, identity standardisation.  Device memory is allocated on first
 * use. */
tpl_mlp *tpl_mlp_create(int in, int hidden, int out, uint64_t seed);
/* hipStream_t for the network's own calls (NULL: the null stream). */
int tpl_mlp_set_stream(tpl_mlp *m, void *hip_stream);
/* Keys: nparams in hidden out adam_steps. */
int tpl_mlp_query(const tpl_mlp *m, const char *key, double *out);
/* FP32 master parameters to / from a host array of exactly nparams floats.
 * Setting them also resets Adam's moments and step count. */
int tpl_mlp_get_params(tpl_mlp *m, float *host, size_t n);
int tpl_mlp_set_params(tpl_mlp *m, const float *host, size_t n);
/* Standardisation (host arrays): the network sees (x - in_mean) / in_std
 * and its outputs are y * out_std + out_mean; scales must be > 0. */
int tpl_mlp_set_norm(tpl_mlp *m, const float *in_mean, const float *in_std,
                     const float *out_mean, const float *out_std);
/* Y[n][out] = network(X[n][in]) in physical units.  X and Y are device
 * pointers (FP32); synchronises before returning. */
int tpl_mlp_forward(tpl_mlp *m, const float *X, float *Y, int64_t n);
/* Gradients of the loss over the n rows of X and T (device, FP32, T raw
 * targets [n][out]) into the host array dW (nparams floats, the flat layout);
 * the loss into *loss if non-NULL.  Parameters are not changed. */
int tpl_mlp_grads(tpl_mlp *m, const float *X, const float *T, int64_t n,
                  float *dW, float *loss);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, learning rate lr) on the
 * loss over the n rows; *loss (if non-NULL) receives the loss before it. */
int tpl_mlp_train_step(tpl_mlp *m, const float *X, const float *T, int64_t n,
                       float lr, float *loss);
void tpl_mlp_destroy(tpl_mlp *m);

/* Coarse state := full-weighting restriction of the fine state: coarse node
 * (X, Y) averages fine nodes (m X + i, m Y + j), |i|, |j| <= m/2, with weight
 * 1/2 on the window's edges (m = nx_fine / nx_coarse = ny_fine / ny_coarse,
 * even), applied to both species' populations and the lagged psi and U; the
 * other per-node fields are recomputed.  Both contexts initialised, FP64
 * storage, same nq. */
int tpl_restrict(const tpl_ctx *fine, tpl_ctx *coarse);
/* Raw features of the current state into the device array X [nx ny][54]:
 * feature 6 s + f is field f of (rho, Ux, Uy, Cxx, Cxy, Cyy) at stencil
 * position s = 3 (dy + 1) + (dx + 1) (periodic). */
int tpl_features(tpl_ctx *ctx, float *X, size_t len);
/* Targets into the device array T [nx ny][5]: (rho Ux, rho Uy, tau_xx,
 * tau_xy, tau_yy) of the device observables obs_ref ([TPL_NFIELDS][ny][nx],
 * as tpl_moments_device writes them) minus those of the current state. */
int tpl_targets(tpl_ctx *ctx, const double *obs_ref, float *T, size_t len);
/* Extra body force F[2][ny][nx] (host doubles, len = 2 nx ny) added to the
 * forcing of every later step; NULL removes it.  TPL_ESTATE while a network
 * is attached. */
int tpl_set_source(tpl_ctx *ctx, const double *F, size_t len);
/* The extra body force of the last step (zeros if none), host doubles. */
int tpl_get_source(tpl_ctx *ctx, double *F, size_t len);
/* Attach a correction network (in = 54, out = 5) to a context: before every
 * later tpl_step step the library computes the features, the network's
 * correction and the source F from the current state.  Drift gate: if
 * max |F| / rho exceeds drift_bound u0 (the velocity change the correction
 * would make in one step), tpl_step returns TPL_EREJECTED before that step
 * (the state stays at the last completed step).  m = NULL detaches.  The
 * network must outlive the attachment. */
int tpl_attach_mlp(tpl_ctx *ctx, tpl_mlp *m, double drift_bound);

/* Thread-local description of the last error ("" if none). */
const char *tpl_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
