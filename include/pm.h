/*
 * pm.h - C ABI of the MI355X discrete-Green FFT solver for 2D
 * elastic-perfectly plastic, pixelwise disordered porous media
 * (Willot & Pellegrini, arXiv:0802.2488).
 *
 * The problem (Sec. 2, first paragraph; eq. 1): an L x L periodic lattice of
 * pixels, each either a void (stress free) or an elastic-perfectly plastic
 * Mises matrix element with flow stress Y under deformation theory; strains
 * are forward differences of a periodic displacement, equilibrium uses
 * backward differences; an overall strain E is prescribed and increased step
 * by step (Sec. 2, end of "Discrete Green functions").  The solver is the
 * augmented-Lagrangian Lippmann-Schwinger FFT iteration (Sec. 1) with the
 * discrete Green tensor of eq. 3 and the convergence indicators of Sec. 2,
 * "Convergence issues".
 *
 * Conventions of every entry point
 *   - All functions are extern "C", never throw, and return an int status
 *     (PM_OK = 0 or a negative PM_E* code).  pm_last_error() then returns a
 *     thread-local message for the last failing call of the thread.
 *   - Device pointers are HIP device memory of the current device; host
 *     pointers are ordinary host memory.  The library never allocates device
 *     memory: the caller provides the workspace (pm_workspace_bytes) and all
 *     output buffers, and keeps them alive while they are in use.
 *   - "stream" is a hipStream_t passed as void* (NULL = the null stream).
 *     All device work of a solver is issued on its stream.
 *   - Fields are row-major [x2][x1] with x1 (the direction of e^1) the
 *     contiguous index, p = x2 * L + x1.  Tensor fields are stored as planes
 *     of L*L values in the order 11, 22, 33, 12 (tensor components; the
 *     shear plane holds eps_12, not the engineering strain 2 eps_12).
 *   - Precision: PM_FP32 keeps fields and FFTs in float and every norm,
 *     mean and convergence test in double; PM_FP64 is double throughout.
 *     Output planes use the field precision.
 */
#ifndef PM_H
#define PM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define PM_OK 0
#define PM_EINVAL (-1)  /* invalid argument: L, moduli, tolerances, pointers, workspace size */
#define PM_EDEVICE (-3) /* a HIP runtime call failed */
#define PM_ENOCONV (-4) /* step stopped at max_iter; outputs are written and valid as iterates */
#define PM_ENAN (-5)    /* a non-finite value reached the FP64 reductions; outputs are written */
#define PM_EBUSY (-6)   /* batch/serving pool cannot admit the request now */

#define PM_FP32 0
#define PM_FP64 1

/* Supported grid sizes: L a power of two with 4 <= L <= PM_MAX_L. */
#define PM_MAX_L 8192

/*
 * Solver parameters.
 *   L                grid side, power of two in [4, PM_MAX_L].
 *   mu, lambda       Lame moduli of the matrix (3-D isotropic; mu > 0,
 *                    3 lambda + 2 mu > 0).
 *   Y                flow stress (Mises norm of the stress in plastic zones, Y > 0).
 *   mu0, lambda0     reference medium of the Green tensor and penalty of the
 *                    augmented Lagrangian (eq. 3, "reference medium of Lame
 *                    moduli mu and lambda"); 0 selects twice the matrix moduli.
 *                    Must satisfy mu0 > 0 and lambda0 + mu0 > 0.
 *   eta_eq           tolerance on the equilibrium indicator eta_1
 *                    (<|div sigma|^2>^(1/2) / |<sigma>|), Sec. 2.
 *   eta_mac          tolerance on eta_2 (change of <sigma> between iterations).
 *   eta_cmp          tolerance on the augmented-Lagrangian constraint
 *                    <|e - eps|^2>^(1/2) / |E|.  A step converges at the first
 *                    iteration >= 2 where all three hold.
 *   max_iter         iteration cap per load step (>= 1).
 *   check_every      iterations issued between host polls of the device
 *                    convergence flag (0 = automatic).  The test itself runs
 *                    on the device at every iteration, so results do not
 *                    depend on this value.
 *   precision        PM_FP32 or PM_FP64.
 *   green_variant    0: G(q1, q2) of eq. 3; 1: G(-q1, -q2); 2: G(-q1, q2);
 *                    3: G(q1, -q2) (the four tensors of the DG2 scheme);
 *                    4: DG1, the symmetrised tensor
 *                    {G(q1,q2) + G(-q1,-q2) + (-1)^(i+j+k+l) [G(-q1,q2) +
 *                    G(q1,-q2)]} / 4 (Sec. 2); 5: CG1, the continuum
 *                    operator -Gamma0 at the continuum frequencies of the
 *                    bins, no strain on modes with a Nyquist component
 *                    (Sec. 2).  4 and 5 run in the single solver only
 *                    (pm_batch_admit rejects them).
 */
typedef struct pm_params {
  int32_t L;
  double mu, lambda, Y;
  double mu0, lambda0;
  double eta_eq, eta_mac, eta_cmp;
  int32_t max_iter;
  int32_t check_every;
  int32_t precision;
  int32_t green_variant;
} pm_params;

/*
 * Per-step outputs.  Device pointers may be NULL to skip that output.
 *   sigma    device, 4 planes (11, 22, 33, 12): S(eps), exactly 0 on voids.
 *   eps      device, 4 planes: the pointwise strain of the last iteration
 *            (eps_33 -> 0 at convergence; arbitrary but finite in voids).
 *   plastic  device uint8 L*L: 1 on matrix pixels whose Mises stress equals
 *            Y (Sec. 3, plastic phase), read from sigma within a tolerance
 *            of 4e-6 Y (FP32) / 1e-12 Y (FP64): the capped branch of the
 *            Mises law except for elastic pixels that close to yield.
 *   host results: <sigma>, <eps> (11, 22, 33, 12), final indicators,
 *   iterations of this step, converged flag, and the step status code.
 */
typedef struct pm_step_out {
  void* sigma;
  void* eps;
  uint8_t* plastic;
  double sigma_mean[4];
  double eps_mean[4];
  double res_eq, res_mac, res_cmp;
  int32_t iters;
  int32_t converged;
  int32_t status;
} pm_step_out;

typedef struct pm_solver pm_solver;

/* Human-readable text for a status code (static storage). */
const char* pm_status_string(int status);

/* Message of the last failing call on this thread ("" if none). */
const char* pm_last_error(void);

/*
 * Bytes of device workspace a solver with these parameters needs
 * (strain state, half spectrum, twiddle and momentum tables, FP64 partials,
 * device convergence state).  Returns 0 if the parameters are invalid.
 */
size_t pm_workspace_bytes(const pm_params* params);

/*
 * Create a solver for one realization.
 *   out          receives the handle (host memory).
 *   params       copied; see pm_params.
 *   d_void_mask  device uint8 L*L, 1 = void (Sec. 2, pixels are voids with
 *                concentration f), any alignment, borrowed until
 *                pm_solver_destroy and not to be changed meanwhile (the state
 *                written from it on the first step keeps the void flags the
 *                iterations use).
 *   d_workspace  device memory of at least pm_workspace_bytes(params),
 *                256-byte aligned, borrowed until pm_solver_destroy.
 *   stream       hipStream_t for all work of this solver.
 * The handle is bound to one stream and is not thread safe.  The first
 * pm_solver_step starts from eps = E, lambda = S(E) on matrix pixels.
 * Errors: PM_EINVAL (parameters, NULL pointers, small or misaligned
 * workspace), PM_EDEVICE.
 */
int pm_solver_create(pm_solver** out, const pm_params* params, const uint8_t* d_void_mask, void* d_workspace,
                     size_t workspace_bytes, void* stream);

/*
 * One load step at overall strain E = (E11, E22, E12), E33 = 0 (plane
 * strain), continuing from the state of the previous step (only the mean
 * strain changes).  Iterates on the device until converged or max_iter,
 * then writes the requested outputs and fills the host fields of *out.
 * E = 0 gives the zero solution with iters = 0 and resets the state.
 * Returns PM_OK on convergence, PM_ENOCONV or PM_ENAN with outputs written,
 * PM_EINVAL or PM_EDEVICE on errors.  Blocks until the step is done.
 */
int pm_solver_step(pm_solver* solver, const double E[3], pm_step_out* out);

/* Release the handle (not the borrowed mask or workspace). */
int pm_solver_destroy(pm_solver* solver);

/* Change the iteration limit of the following load steps (the state is
 * kept), e.g. to replay another solve's iteration counts step by step.
 * Synchronises the solver's stream.  Errors: PM_EINVAL (NULL solver,
 * max_iter < 1). */
int pm_solver_set_max_iter(pm_solver* solver, int32_t max_iter);

/*
 * Fill dst (device if on_device != 0, else host) with the Bernoulli void
 * mask of Sec. 2: pixel p = x2 * L + x1 is a void (1) iff
 * (splitmix64(seed ^ splitmix64(p)) >> 11) * 2^-53 < f, where splitmix64 is
 * the SplitMix64 output function.  L in [1, 65536]; 0 <= f <= 1.
 */
int pm_bernoulli_mask(uint8_t* dst, int32_t L, double f, uint64_t seed, int32_t on_device, void* stream);

/*
 * Tile width WT of the internal half spectrum for this size and precision
 * (negative PM_EINVAL on invalid arguments).  The half spectrum holds, per
 * component c (0: 11, 1: 22, 2: 12), L/2 columns m1 = 0..L/2-1 of L rows
 * m2 = 0..L-1 of complex values in the field precision, at complex index
 *     (((m1 / WT) * L + m2) * WT + m1 % WT) * 3 + c.
 * Row transforms of real fields have real bins m1 = 0 and m1 = L/2; column
 * m1 = 0 stores bin 0 in its real part and bin L/2 in its imaginary part.
 * After a column transform that column holds the transform of that packed
 * complex sequence.
 */
int32_t pm_spectrum_tile(int32_t L, int32_t precision);

/*
 * Kernel-level entry points on a solver's own buffers (used to check each
 * kernel in isolation), with the half spectrum in the layout of
 * pm_spectrum_tile.
 *
 * pm_solver_buffers   device pointers of the solver state and of the half
 *                     spectrum.  The state is the stress of the last iterate,
 *                     (11, 22, 33, 12) of each pixel side by side, pixels
 *                     x2-major (a void's stress is zero, its 33 component a
 *                     negative zero, which marks the void for the iteration
 *                     pass; outputs carry +0); it is also the augmented-Lagrangian
 *                     multiplier; the strain is recovered from it and the
 *                     stored polarisation when outputs are written.
 * pm_debug_forward    d_real: 3 planes (11, 22, 12).  Spectrum := the 2-D
 *                     DFT sum_x f(x) exp(-i q.x) of each plane (packed
 *                     column 0 as described above).
 * pm_debug_inverse    d_real := the unnormalised inverse 2-D DFT
 *                     sum_q F(q) exp(+i q.x) of the Hermitian-extended
 *                     spectrum (L^2 times numpy.fft.irfft2); the spectrum
 *                     buffer is overwritten.
 * pm_debug_green      spectrum(q) := G(q):spectrum(q) (eq. 3, built from
 *                     mu0, lambda0, green_variant) for q != 0 and E at q = 0;
 *                     column 0 is split into its m1 = 0 and m1 = L/2 parts by
 *                     conjugate symmetry in m2, each gets its own tensor, and
 *                     the results are packed again.
 * All three issue work on the solver's stream and synchronise it.
 */
int pm_solver_buffers(pm_solver* solver, void** d_state, void** d_spectrum);

/*
 * Per-kernel device time of the iterations a solver has run while timing was
 * on, from HIP events recorded on the solver's stream around each launch.
 *   col_ms / col_launches      column pass (FFT, Green tensor, inverse FFT)
 *   row_ms / row_launches      row pass (inverse FFT, pointwise step, FFT)
 *   other_ms                   reductions and equilibrium residual
 * Only iterations that did work are counted (launches after convergence
 * exit at once and are excluded).
 */
typedef struct pm_kernel_timing {
  double col_ms;
  int64_t col_launches;
  double row_ms;
  int64_t row_launches;
  double other_ms;
  int64_t iterations;
} pm_kernel_timing;

/*
 * enable = n >= 1 resets the totals and starts timing every n-th iteration
 * (events around its launches; each event pair costs device time, so a
 * sampled n keeps the timed run close to an untimed one); 0 stops timing.
 * Host polling stays pipelined: a chunk's events are read once its state
 * has come back.  out (may be NULL) receives the totals accumulated so far.
 * Errors: PM_EINVAL (NULL solver, enable < 0), PM_EDEVICE.
 */
int pm_solver_timing(pm_solver* solver, int32_t enable, pm_kernel_timing* out);
int pm_debug_forward(pm_solver* solver, const void* d_real);
int pm_debug_inverse(pm_solver* solver, void* d_real);
int pm_debug_green(pm_solver* solver, const double E[3]);


/* ------------------------------------------------------------------------
 * Batch / serving engine.
 *
 * Many independent realizations, each with its own mask, moduli, grid size,
 * precision and load ramp E_1..E_n, solved together on one stream: every
 * launch covers all running realizations ("slots") of one (precision, L)
 * group, and each slot advances along its own ramp on the device, the state
 * of one load step warm-starting the next exactly as successive calls of
 * pm_solver_step do (the solved problem is the one of eqs. 1-3 with the
 * pointwise law of Sec. 2; the load ramp is the stepwise strain history of
 * Sec. 3).  A slot's step records and fields are bitwise identical to those
 * of a pm_solver with the same parameters driven through the same ramp: the
 * kernels and the fixed-order reductions are the same, per slot.
 *
 * Memory: the caller passes one device pool.  The engine keeps its fixed
 * part (pm_batch_overhead_bytes) at the start of the pool and carves each
 * slot's workspace (pm_batch_slot_bytes) out of the rest, first fit; it
 * never allocates device memory.  Admission fails with PM_EBUSY when the
 * pool has no free range of that size or all max_slots slots are in use.
 *
 * Threading: a pm_batch is bound to its stream and is not thread-safe.
 * Masks passed to pm_batch_admit must stay alive until pm_batch_release.
 * ---------------------------------------------------------------------- */
typedef struct pm_batch pm_batch;

/* One load step's result, written by the device when the step ends. */
typedef struct pm_step_record {
  double sigma_mean[4];      /* <sigma> 11, 22, 33, 12 (FP64) */
  double eps_mean[4];        /* <eps> of the recovered strain */
  double res_eq, res_mac, res_cmp;
  double plastic_fraction;   /* pixels on the capped branch in the last iteration / L^2 */
  int32_t iters;
  int32_t status;            /* 1 converged, 2 stopped at max_iter, 3 non-finite value */
} pm_step_record;

#define PM_STEP_CONVERGED 1
#define PM_STEP_NOCONV 2
#define PM_STEP_NAN 3

/* State of a slot as of the end of the last pm_batch_tick. */
typedef struct pm_slot_info {
  int32_t L, precision, nsteps;
  int32_t steps_done;        /* records 0 .. steps_done-1 are final */
  int32_t finished;          /* 1: all steps done, or stopped at a non-finite value */
  int32_t last_status;       /* status of the last finished step (0 if none) */
  int32_t held;              /* 1: waiting after step steps_done-1 (PM_ADMIT_HOLD) */
} pm_slot_info;

/* Admission flag: after each load step (but the last) the slot waits with the
 * converged fields of that step until pm_batch_resume; pm_batch_fetch then
 * returns exactly that step's fields.  Used to combine several slots step by
 * step (DG2). */
#define PM_ADMIT_HOLD 1

/* Fixed part of the pool for max_slots slots (slot states, the device slot
 * table and the twiddle / momentum tables of every grid size). */
size_t pm_batch_overhead_bytes(int32_t max_slots);

/* Pool bytes one slot with these parameters and nsteps load steps takes
 * (state, half spectrum, partial sums, ramp and step records); 0 if params
 * are invalid. */
size_t pm_batch_slot_bytes(const pm_params* params, int32_t nsteps);

/* d_pool: device memory of pool_bytes bytes, 256-byte aligned, owned by the
 * caller and kept alive until pm_batch_destroy.  1 <= max_slots <= 65536. */
int pm_batch_create(pm_batch** out, void* d_pool, size_t pool_bytes, int32_t max_slots, void* stream);

/* Admit a realization.  d_void_mask: device, L x L row-major [x2][x1],
 * 1 = void.  E_path: host, nsteps x 3 (E11, E22, E12 per step, each of
 * nonzero finite norm), copied.  On success *slot receives the slot id.
 * The first step starts from the uniform state of that step's E (as the
 * first pm_solver_step).  The work is queued on the batch's stream; it
 * runs with the next ticks.  flags: 0 or PM_ADMIT_HOLD.  Returns PM_EBUSY
 * (nothing changed) when the pool or the slot table is full. */
int pm_batch_admit(pm_batch* batch, const pm_params* params, const uint8_t* d_void_mask, int32_t nsteps,
                   const double* E_path, int32_t flags, int32_t* slot);

/* Start the next load step of a slot admitted with PM_ADMIT_HOLD that is
 * waiting (pm_slot_info.held); queued on the batch's stream.  PM_EINVAL if
 * the slot is not waiting. */
int pm_batch_resume(pm_batch* batch, int32_t slot);

/* Run iters augmented-Lagrangian iterations on every running slot, then end
 * the load steps that finished (output pass for <eps>, record, start of the
 * next step), then read back every slot's state (blocking).  A slot whose
 * step ends during a tick waits for the end of that tick.  *running (may be
 * NULL) receives the number of slots not finished. */
int pm_batch_tick(pm_batch* batch, int32_t iters, int32_t* running);

int pm_batch_poll(pm_batch* batch, int32_t slot, pm_slot_info* info);

/* Copy step records first .. first+count-1 (all < steps_done) to host. */
int pm_batch_records(pm_batch* batch, int32_t slot, int32_t first, int32_t count, pm_step_record* out);

/* Write the slot's current fields (sigma, eps, plastic mask; device
 * pointers of pm_step_out, NULL = skip) and means, as pm_solver_step does
 * after a step.  Meaningful once steps_done > 0; blocking. */
int pm_batch_fetch(pm_batch* batch, int32_t slot, pm_step_out* out);

/* Free the slot's pool range and id.  A slot that is still running is
 * stopped.  Blocking (waits for queued work). */
int pm_batch_release(pm_batch* batch, int32_t slot);
int pm_batch_destroy(pm_batch* batch);

/* enable = 1 (the default): once a slot table has run one tick eagerly, the
 * launches of later ticks with that table and iteration count are captured
 * into a HIP graph and replayed; 0 launches every tick eagerly.  Results do
 * not depend on it.  The engine works on a stream of its own (default
 * priority), ordered after the caller's stream at every call. */
int pm_batch_set_graphs(pm_batch* batch, int32_t enable);


/* ------------------------------------------------------------------------
 * DG2 (Sec. 2, "Discrete Green functions"): the same system is solved to
 * convergence with the Green tensor of eq. 3 taken at (q1, q2), (-q1, -q2),
 * (-q1, q2) and (q1, -q2) (green_variant 0..3), and the four strain fields
 * are averaged.  pm_dg2_combine forms, per pixel, the average strain, the
 * Hencky-Mises stress of the average (zero on voids), the average of the
 * four stresses and the plastic mask of the average (matrix pixels with
 * 3 mu eps_eq > Y), and the FP64 means of the three fields.
 * ---------------------------------------------------------------------- */
typedef struct pm_dg2_out {
  void* eps;               /* device, 4 planes (11, 22, 33, 12), or NULL */
  void* sigma_of_avg;      /* device, 4 planes, or NULL */
  void* sigma_avg;         /* device, 4 planes, or NULL (needs d_sigma) */
  uint8_t* plastic;        /* device, L x L, or NULL */
  double eps_mean[4];
  double sigma_of_avg_mean[4];
  double sigma_avg_mean[4];   /* zeros when d_sigma is NULL */
  double plastic_fraction;
} pm_dg2_out;

/* Device workspace pm_dg2_combine needs for these parameters (partial sums);
 * 0 if params are invalid. */
size_t pm_dg2_workspace_bytes(const pm_params* params);

/* params: L, mu, lambda, Y and precision of the four solves.  d_eps[v],
 * d_sigma[v]: device fields (4 planes each, field precision) of variant v;
 * d_sigma may be NULL.  Queued on stream, then synchronised for the means.
 * Inputs and outputs may not overlap. */
int pm_dg2_combine(const pm_params* params, const uint8_t* d_void_mask, const void* const d_eps[4],
                   const void* const d_sigma[4], void* d_workspace, size_t workspace_bytes, pm_dg2_out* out,
                   void* stream);

/* pm_dg2_combine without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, serving loops,
 * harnesses that forbid hipMalloc).  It allocates nothing: its partial sums
 * live in a static device array of pm_dg2_combine_static_max_bytes() bytes
 * (about 131 KB; one copy on every GPU the library runs on, held until the
 * process ends), which covers every L up to PM_MAX_L.  Arguments, outputs,
 * results and errors as pm_dg2_combine (PM_EINVAL also when an input would
 * need more scratch than the array holds).  All calls on one GPU share the
 * array: calls that overlap in time on one GPU (other host threads, other
 * streams) race and must be serialised by the caller. */
size_t pm_dg2_combine_static_max_bytes(void);
int pm_dg2_combine_static(const pm_params* params, const uint8_t* d_void_mask, const void* const d_eps[4],
                          const void* const d_sigma[4], pm_dg2_out* out, void* stream);


/* ------------------------------------------------------------------------
 * Void and plastic clusters (Sec. 3).  Phases: void (mask 1), plastic
 * (matrix pixels of a plastic mask, e.g. the output of a step) and elastic.
 * Clusters are periodic nearest-neighbour (4-connected) components; the
 * void-plastic phase is the union of voids and plastic pixels, and a plastic
 * cluster that touches no void is joined to the cluster of its nearest void
 * pixel (periodic Euclidean distance, ties to the smaller pixel index).
 * Labels are canonical: a cluster's label is its smallest pixel index
 * x2 * L + x1; elastic pixels get -1.
 * ---------------------------------------------------------------------- */
typedef struct pm_cluster_stats {
  int64_t n_void, n_plastic;        /* pixels (plastic counts matrix pixels only) */
  int64_t n_void_clusters;          /* clusters of the void phase alone */
  int64_t n_clusters_raw;           /* void-plastic clusters before attachment */
  int64_t n_isolated_void_clusters; /* of those, clusters without plastic pixels */
  int64_t n_plastic_only_clusters;  /* of those, clusters without voids (attached when voids exist) */
  int64_t n_clusters;               /* void-plastic clusters after attachment */
  int64_t largest;                  /* pixels of the largest cluster (ties: smallest label) */
  int32_t largest_label;            /* its label, -1 if there is no cluster */
  int32_t spans_x1, spans_x2;       /* the largest cluster holds a pixel in every column / row */
  int32_t pad;
} pm_cluster_stats;

/* Device workspace of pm_clusters (about 12 bytes per pixel); 0 if L is invalid. */
size_t pm_cluster_workspace_bytes(int32_t L);

/* d_void_mask, d_plastic: device L x L uint8 (nonzero = void / plastic).
 * d_labels: device L x L int32, receives the labels.  Work is queued on
 * stream; the call synchronises it to return the counts. */
int pm_clusters(int32_t L, const uint8_t* d_void_mask, const uint8_t* d_plastic, int32_t* d_labels,
                void* d_workspace, size_t workspace_bytes, pm_cluster_stats* out, void* stream);

/* Per-step indicators of Sec. 3 (Fig. 2 legend) from the counts of one
 * pm_clusters call on an L x L grid:
 *   v_p   = (void + plastic pixels) / L^2, the void-plastic volume fraction;
 *   f_p   = v_p / (1 - f), its normalised form, with f = void_fraction, or
 *           the realised n_void / L^2 when void_fraction < 0;
 *   v_max = pixels of the largest void-plastic cluster / L^2;
 *   i     = void clusters holding no plastic pixel / void clusters (the
 *           proportion of isolated voids);
 *   n     = void-plastic clusters after the nearest-void attachment / void
 *           clusters (at zero load every void-plastic cluster is a void
 *           cluster, so n is normalised to its value there).
 * With no void cluster, i and n divide by 1.  Host memory only; errors:
 * PM_EINVAL (NULL pointer, L not a power of two in [4, PM_MAX_L], counts
 * negative or beyond L^2, f >= 1). */
typedef struct pm_cluster_indicators_out {
  double v_p, f_p, v_max, i, n;
} pm_cluster_indicators_out;

int pm_cluster_indicators(const pm_cluster_stats* stats, int32_t L, double void_fraction,
                          pm_cluster_indicators_out* out);

/* Loading-path indicators of Sec. 3 (r = dn/d eps0, and -d2 sigma0/d eps0^2
 * from the mean stress curve): first and second derivatives of samples
 * y[k] taken at strictly increasing x[k], k < n_steps, by three-point
 * finite differences on the non-uniform grid (central inside, one-sided at
 * the ends; exact for quadratics).  All arrays are host memory of n_steps
 * doubles; dy or d2y may be NULL.  Errors: PM_EINVAL (n_steps < 3, NULL x
 * or y, x not strictly increasing or not finite). */
int pm_path_derivatives(int32_t n_steps, const double* x, const double* y, double* dy, double* d2y);


/* Measures of a strain map, for the comparison of the methods in Sec. 2
 * (Fig. 1: checkerboard patterns of CG1 and CG2, blurring by DG1).  On the
 * matrix pixels (mask 0) of an L x L strain field d_eps (device, 4 planes
 * 11, 22, 33, 12 of the given precision), with eps_eq = [(2/3) e':e']^(1/2)
 * and e' the 3-D deviator (Fig. 1):
 *   mean_eq, max_eq   mean and maximum of eps_eq;
 *   checkerboard      root mean square of the mixed second difference
 *                     eps_eq(x) - eps_eq(x+e1) - eps_eq(x+e2) + eps_eq(x+e1+e2)
 *                     over 2 x 2 blocks of matrix pixels, divided by mean_eq
 *                     (0 for a field varying along one axis; 4 b / a for
 *                     eps_eq = a + b (-1)^(x1+x2));
 *   sharpness         root mean square of the differences between matrix
 *                     nearest neighbours, divided by mean_eq.
 * Periodic neighbours; FP64 sums in a fixed order.  The workspace holds the
 * partial sums (pm_strain_map_workspace_bytes, 8-byte aligned).  Queued on
 * stream, then synchronised.  Errors: PM_EINVAL (L, precision, NULL or
 * small workspace). */
typedef struct pm_strain_map_out {
  double mean_eq, max_eq, checkerboard, sharpness;
  int64_t matrix_pixels;
} pm_strain_map_out;

size_t pm_strain_map_workspace_bytes(int32_t L);
int pm_strain_map_metrics(int32_t L, int32_t precision, const void* d_eps, const uint8_t* d_void_mask,
                          void* d_workspace, size_t workspace_bytes, pm_strain_map_out* out, void* stream);

/* CG2 (Sec. 2): the average of a field over each pixel and its four nearest
 * neighbours (periodic), applied plane by plane.  d_in, d_out: device,
 * nplanes x L x L values of the given precision, not overlapping.  Queued
 * on stream (not synchronised). */
int pm_five_point_average(int32_t L, int32_t precision, int32_t nplanes, const void* d_in, void* d_out,
                          void* stream);


/* ------------------------------------------------------------------------
 * Autotuning.  For each (precision, L) the iteration kernels exist in two
 * variants: the row pass with another FFT radix, and the column pass with
 * another radix (and columns per block).  The data layout is the same for
 * all variants.  The choice is process-wide and read at every iteration by
 * solvers and batches; results of a solve depend on it only through
 * rounding.  Change it between solves, not during them.
 * ---------------------------------------------------------------------- */
typedef struct pm_tune_result {
  int32_t row_variant, col_variant;    /* the fastest, now in effect */
  double ms_per_iteration[2][2];       /* measured [row][col] */
} pm_tune_result;

/* Device workspace pm_autotune needs (a solver's workspace and a mask). */
size_t pm_autotune_workspace_bytes(int32_t L, int32_t precision);

/* Time iters iterations of every variant pair on a synthetic grid (voids
 * f = 0.2, material mu = 1, lambda = 2, Y = 1) and put the fastest into
 * effect for (L, precision).  Blocking. */
int pm_autotune(int32_t L, int32_t precision, int32_t iters, void* d_workspace, size_t workspace_bytes,
                void* stream, pm_tune_result* out);
int pm_set_tuning(int32_t L, int32_t precision, int32_t row_variant, int32_t col_variant);
int pm_get_tuning(int32_t L, int32_t precision, int32_t* row_variant, int32_t* col_variant);

#ifdef __cplusplus
}
#endif

#endif /* PM_H */
