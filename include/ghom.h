/*
 * ghom.h -- C ABI of libghom.so: Galerkin-FFT homogenization with macroscopic stress,
 * deformation-gradient or mixed control, on one AMD Instinct MI355X (gfx950).
 *
 * Method: S. Lucarini, J. Segurado, "An algorithm for stress and mixed control in
 * Galerkin based FFT homogenization", arXiv:1901.06531.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - A tensor field is 9 contiguous planes of N = nx*ny*nz values (C order, z fastest):
 *    value (c, x, y, z) sits at c*N + (x*ny + y)*nz + z, component c = 3*i + j holding the
 *    tensor entry (i, j).  This is a NumPy array of shape (9, nx, ny, nz).
 *  - Scalar per-voxel fields (phase, stiffness scale) are single planes of N values.
 *  - A control mask is 9 bytes: mask[c] = 1 prescribes the macroscopic first
 *    Piola-Kirchhoff stress component c (the paper's IJ terms, Sec. 2.3), mask[c] = 0
 *    prescribes the macroscopic deformation-gradient component c (ij terms).
 *  - Host pointers ("host") are read or written synchronously and stay owned by the
 *    caller; the library copies what it keeps.  Device pointers ("dev") are HIP device
 *    memory owned by the caller, accessed on the context's stream; the call returns after
 *    the stream has finished with them.
 *  - Every call returns GHOM_OK (0) or a negative status; it never throws.  The message
 *    of the last failure of a context is returned by ghom_last_error.
 *  - One context per host thread and stream.  All device memory of a context is
 *    allocated by ghom_create and released by ghom_destroy.
 */
#ifndef GHOM_H
#define GHOM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ghom_ctx ghom_ctx;

/* Arithmetic of the conjugate-gradient solve.
 *  GHOM_FP64       : everything in float64.
 *  GHOM_FP32_SPLIT : CG vectors, tangent state and the transforms inside CG in float32
 *                    with float64 dot products; F, P, the Newton residual, the averages
 *                    and a float64 re-projection of every Newton correction in float64.
 *                    Each CG solve stops no tighter than 1e-5 of its right-hand side (the
 *                    cg_forcing of ghom_set_tolerances is raised to 1e-5 at least): float32
 *                    CG cannot go much further, and the float64 Newton iteration reaches
 *                    the Newton tolerance regardless. */
enum { GHOM_FP64 = 0, GHOM_FP32_SPLIT = 1 };

enum {
  GHOM_OK = 0,
  GHOM_EINVAL = -1,         /* bad argument (message says which)                          */
  GHOM_ENOMEM = -2,         /* device allocation failed                                    */
  GHOM_EHIP = -3,           /* a HIP runtime call or kernel launch failed                  */
  GHOM_ENOTCONVERGED = -4,  /* Newton or CG iteration cap; fields hold the last iterate    */
  GHOM_ESINGULAR = -5,      /* CG breakdown at its first iteration (p.Ap <= 0)             */
  GHOM_EDOMAIN = -6,        /* det F <= 0 at some voxel                                    */
  GHOM_ESTATE = -7          /* call order: e.g. step before material, control or history   */
};

/* Fields readable with ghom_get_field / ghom_get_field_device. */
enum { GHOM_FIELD_F = 0, GHOM_FIELD_P = 1 };

/* Outcome of one load increment (ghom_step) or one Newton solve. */
typedef struct {
  int newton_iters;    /* Newton iterations (residual evaluations)                         */
  int cg_iters_total;  /* conjugate-gradient iterations summed over the Newton iterations   */
  int cg_breakdowns;   /* CG solves stopped early by p.Ap <= 0 after their first iteration */
  int status;          /* the call's return value                                          */
  double crit;         /* last Newton criterion max_x |dF(x)| / |<F>|                      */
  double res_rms;      /* voxel-averaged L2 norm of the last Newton residual               */
  double t_total_ms;   /* wall time of the call                                            */
  double t_cg_ms;      /* time inside the CG loops                                         */
  int cg_stalls;       /* CG solves stopped because r.r found no new minimum in 20
                          iterations (a residual floor above the threshold); Newton goes on
                          with the iterate                                                  */
  int reserved;
} ghom_step_info;

/* Creates a context for an nx x ny x nz voxel grid of the periodic cell of edge lengths
 * (Lx, Ly, Lz) (the frequency vector is xi_d = k_d / L_d, Sec. 2.1 "Projection operator").
 * Each n_d must be one of 4, 6, 8, 9, 12, 16, 18, 24, 27, 32, 36, 48, 64, 72, 96, 128, 144,
 * 192, 256, 512.  precision: GHOM_FP64 or GHOM_FP32_SPLIT.  device: HIP device index.
 * hip_stream: a hipStream_t to run on (e.g. torch's current stream), or NULL for a new
 * stream owned by the context.  On success *out receives the context. */
int ghom_create(ghom_ctx **out, int nx, int ny, int nz, double Lx, double Ly, double Lz,
                int precision, int device, void *hip_stream);

/* Releases the context and all its device memory (NULL is ignored). */
void ghom_destroy(ghom_ctx *ctx);

/* Message of the last failed call on ctx ("" if none); valid until the next call.  With
 * ctx NULL: the reason the last ghom_create or ghom_batch_create of this thread failed. */
const char *ghom_last_error(const ghom_ctx *ctx);

/* Compressible neo-Hookean phases: W = mu/2 (tr F^T F - 3) - mu ln J + lam/2 (ln J)^2,
 * P = mu (F - F^-T) + lam ln J F^-T.  phase (host, N values < nphase), mu and lambda
 * (host, nphase values each).  Resets the deformation to F = I and the increment to 0. */
int ghom_set_material_neohookean(ghom_ctx *ctx, const uint16_t *phase, int nphase,
                                 const double *mu, const double *lambda);

/* Saint Venant-Kirchhoff phases (Sec. 3.1): P = F S, S = C : E, E = (F^T F - I)/2.
 * C (host) holds nphase stiffness tensors of 81 values C_ijkl (index ((i*3+j)*3+k)*3+l),
 * each with the minor and major symmetries (checked; EINVAL otherwise).
 * Resets the deformation to F = I and the increment to 0. */
int ghom_set_material_svk(ghom_ctx *ctx, const uint16_t *phase, int nphase, const double *C);

/* Viscoelastic phases: a path- and rate-dependent law with internal variables (the
 * general setting of eq. 1; the paper's own crystal-plasticity model is not given).
 * Saint Venant-Kirchhoff form with one relaxing branch: S = Cinf : E + Q, P = F S, where the
 * overstress Q obeys dQ/dt + Q / tau = C1 : dE/dt.  Over each load increment of length dt
 * (ghom_set_time_step) E is taken linear in time, which integrates exactly to
 * Q = a Q_n + b C1 : (E - E_n), a = exp(-dt/tau), b = tau (1 - a) / dt, with E_n and Q_n the
 * values committed at the end of the previous increment; the Newton tangent is the
 * Saint Venant-Kirchhoff one with the stiffness Cinf + b C1.  Cinf and C1 (host): nphase
 * stiffness tensors of 81 values each, as for ghom_set_material_svk; tau (host): nphase
 * relaxation times > 0.  The internal variables start at zero; a converged (or
 * ENOTCONVERGED) increment commits them.  Resets the deformation to F = I and the increment
 * to 0.  With this law ghom_resolve returns GHOM_EINVAL, ghom_load_state accepts step 0 only
 * (it also zeroes the internal variables), and the batch API does not take it.  The context
 * keeps 12 more float64 planes (E_n, Q_n).  ghom_adjoint_grad_scale works through the whole
 * history when GHOM_OPT_CHECKPOINTS was on from increment 0. */
int ghom_set_material_visco(ghom_ctx *ctx, const uint16_t *phase, int nphase, const double *Cinf,
                            const double *C1, const double *tau);

/* Length of every load increment for rate-dependent laws (default 1; ghom_step_adaptive
 * gives each sub-increment its share).  Must be finite and > 0. */
int ghom_set_time_step(ghom_ctx *ctx, double dt);

/* Per-voxel stiffness scale s(x) > 0 multiplying every modulus of the voxel (host, N
 * values; NULL restores s = 1).  Used by ghom_adjoint_grad_scale. */
int ghom_set_stiffness_scale(ghom_ctx *ctx, const double *s);

/* Control mask of eq. (22) (host, 9 bytes, see above).
 *
 * Rotation gauge of full stress control (GHOM_OPT_ROTATION_GAUGE, on by default): with every
 * component stress-controlled (eq. 19) the deformation gradient is fixed only up to the
 * rigid rotations that leave the prescribed stress unchanged (P(QF) = Q P(F)): all three at a
 * zero target, where the Newton system becomes singular, and the rotation about e_a under a
 * uniaxial target p e_a (x) e_a.  When the mask is all ones and every row of the history is a
 * multiple of e_a (x) e_a for one axis a, the solver holds the entries F_ba, F_ca and F_cb of
 * <F> ((a, b, c) in cyclic order; zero from F = I) in place of the stress components ba, ca,
 * cb.  At equilibrium <P> <F>^T is symmetric (the average of P F^T over a periodic cell with
 * compatible F and divergence-free P, and P F^T is symmetric at each voxel), which with those
 * three entries at zero forces the three released stress components to their target 0: the
 * solution is the full stress one with its rotation fixed.  Any other mask or history is
 * solved as set.  ghom_get_control reports the mask in use. */
int ghom_set_control(ghom_ctx *ctx, const uint8_t mask[9]);

/* The mask the solver uses (host, 9 bytes; nullable) and the axis of the rotation gauge
 * (0..2, or -1 when it does not apply; nullable).  GHOM_ESTATE before ghom_set_control. */
int ghom_get_control(ghom_ctx *ctx, uint8_t mask_out[9], int *gauge_axis);

/* Load history (host, nsteps x 9): row k-1 holds, for increment k, the prescribed
 * P-bar on stress-controlled and F-bar on deformation-controlled components (eq. 21).
 * The deformation-controlled means are moved uniformly by the change of F-bar at each
 * increment (F-bar of increment 0 is the identity). */
int ghom_set_history(ghom_ctx *ctx, int nsteps, const double *target);

/* Stopping rules (Sec. 4): CG stops when the voxel-averaged L2 norm of its residual,
 * sqrt(sum |r|^2 / N), is <= max(cg_tol, cg_forcing * that norm of the right-hand side);
 * Newton stops when max_x |dF(x)| / |<F>| < newton_tol, or when the residual itself is
 * already <= cg_tol.  Defaults: 1e-6, 1e-8, 0, 50, 5000.  GHOM_EINVAL unless
 * newton_tol > 0, cg_tol > 0, 0 <= cg_forcing < 1, max_newton >= 1 and max_cg >= 1. */
int ghom_set_tolerances(ghom_ctx *ctx, double newton_tol, double cg_tol, double cg_forcing,
                        int max_newton, int max_cg);

/* Advances one load increment: shifts the deformation-controlled means, then Newton
 * (eq. 20) with CG on A(dF) = G*(K : dF) and the modified projection of eq. (22).
 * info (nullable, host) receives the iteration counts and timings.  On
 * GHOM_ENOTCONVERGED the fields hold the last iterate; on GHOM_ESINGULAR / GHOM_EDOMAIN
 * the increment counter is not advanced. */
int ghom_step(ghom_ctx *ctx, ghom_step_info *info);

/* Adaptive stepping (the remedy Sec. 4 names for increments that need many Newton
 * iterations): advances one load increment like ghom_step, walking it in sub-increments
 * along which the prescribed values move linearly from those of the current increment to
 * those of the next.  A sub-increment that ends in GHOM_ENOTCONVERGED, GHOM_ESINGULAR or
 * GHOM_EDOMAIN is retried from its starting state with half its length, at most max_cuts
 * times per call (0..30); one that converges within grow_below Newton iterations doubles
 * the next length.  The next call starts with the length the last one ended with
 * (ghom_set_history and ghom_load_state reset it to the whole increment).  info (nullable)
 * sums the iteration counts and CG time of every attempt; *substeps and *cuts (nullable)
 * receive the accepted sub-increments and the retries.  When the cuts run out the call
 * returns the last failure's status, F is restored to its value at the start of the
 * increment and the increment counter is not advanced.  The context keeps two extra
 * float64 fields (2 x 9 x N) for the restart points, allocated at the first call. */
int ghom_step_adaptive(ghom_ctx *ctx, int max_cuts, int grow_below, ghom_step_info *info,
                       int *substeps, int *cuts);

/* Re-solves equilibrium at the current increment without moving the prescribed means
 * (e.g. after ghom_set_stiffness_scale or ghom_load_state).  info as in ghom_step. */
int ghom_resolve(ghom_ctx *ctx, ghom_step_info *info);

/* Voxel averages <F> and <P> of the current state (host, 9 values each, float64): the
 * macroscopic deformation gradient and first Piola-Kirchhoff stress, F-bar and P-bar of
 * Sec. 2.1-2.3 (the mean of a field equals its zero-frequency Fourier coefficient, Sec. 2.2),
 * whose histories are the paper's macroscopic response curves (Sec. 3.1 Fig. 1, Sec. 3.2
 * Fig. 2).  Reduced in float64 in a fixed order (the same bits on every run). */
int ghom_get_averages(ghom_ctx *ctx, double Fbar[9], double Pbar[9]);

/* Copies field `which` (GHOM_FIELD_F or GHOM_FIELD_P, float64, 9 x N, layout above) to host
 * memory: the microscopic deformation gradient F(x) and stress P(F(x)) of Sec. 2.1 at the
 * current state (the unknown of eq. 3-5 and its stress).  GHOM_EINVAL for another `which`.
 * For the elastic laws the Newton iteration does not store P(x) (it needs only its transform
 * and average); the first request after an evaluation computes it from F(x) by one pass over
 * the field, which leaves the averages as they were. */
int ghom_get_field(ghom_ctx *ctx, int which, double *host_out);

/* Same into caller-owned device memory (float64, 9 x N): waits for the context's stream,
 * then copies; returns when the copy has finished. */
int ghom_get_field_device(ghom_ctx *ctx, int which, double *dev_out);

/* Current deformation gradient (host, 9 x N) and increment index: the state a load
 * increment of Sec. 2.1 starts from (eq. 5: F of increment k+1 is sought from the converged F
 * of increment k), so that a history can be resumed or an increment repeated. */
int ghom_save_state(ghom_ctx *ctx, double *F_out, int *step_out);

/* Sets the deformation gradient (host, 9 x N) and the increment index (0..nsteps) -- the
 * converged state of increment `step`, from which the next ghom_step starts (Sec. 2.1).
 * GHOM_EINVAL for a step out of range. */
int ghom_load_state(ghom_ctx *ctx, const double *F_in, int step);

/* Adjoint gradient of J = a : <F> with respect to s(x) at the current (converged) state:
 * solves A lam = G*(a/N) with the same operator, then dJ/ds(x) = -lam(x) : P(x) / s(x).
 * a (host, 9 values), grad_out (host, N values).  For the viscoelastic law (path
 * dependent) J is taken at the end of the history and the gradient runs backward over every
 * checkpointed increment (GHOM_OPT_CHECKPOINTS from increment 0, else GHOM_ESTATE): per
 * increment one CG solve with that increment's operator on G*(F_n (mE + b s C1 : mQ)), where
 * (mE, mQ) carry the sensitivity of the internal variables from the later increments; the
 * end-of-history state is restored afterwards.  Work memory: 43 x N float64. */
int ghom_adjoint_grad_scale(ghom_ctx *ctx, const double a[9], double *grad_out);

/* ---- hot-path entry points on device memory ------------------------------------- */

/* Av = A(v) = G*(K(F) : v) (eq. 20 left-hand side) at the current F.  v and Av are
 * device arrays of 9 x N values of the CG type: float64 (GHOM_FP64) or float32
 * (GHOM_FP32_SPLIT); they must not overlap. */
int ghom_apply_operator(ghom_ctx *ctx, const void *v_dev, void *Av_dev);

/* out = G*(in) (float64 device arrays of 9 x N; in may equal out): the modified
 * projection of eq. (22) with the context's mask, applied through the 3-D transforms. */
int ghom_apply_projection(ghom_ctx *ctx, const double *in_dev, double *out_dev);

/* For callers that cannot allocate device memory (tight serving loops, harnesses that
 * forbid hipMalloc): out = G*(in) as ghom_apply_projection computes it, without a context and
 * without allocating.  The transforms run in a static device array of 24 MiB per GPU, held by
 * every GPU the library runs on until the process ends, so the grid's half spectrum must fit
 * in it: at most 64^3 voxels (a larger grid returns GHOM_EINVAL with the sizes).  nx, ny, nz,
 * Lx, Ly, Lz as in ghom_create; mask (host, 9 bytes) as in ghom_set_control, used as given
 * (no rotation gauge: there is no history); in_dev and out_dev: float64 device arrays of
 * 9 x N on GPU `device` (in may equal out).  hip_stream: the stream to run on (NULL: the null
 * stream).  Returns after the stream has finished.  Every call on one GPU uses the same array
 * and leaves its contents behind: calls that overlap on one GPU (other threads or streams)
 * race and must be serialized by the caller.  Errors: GHOM_EINVAL, GHOM_EHIP; the message is
 * ghom_last_error(NULL). */
int ghom_apply_projection_static(int nx, int ny, int nz, double Lx, double Ly, double Lz,
                                 const uint8_t mask[9], const double *in_dev, double *out_dev,
                                 int device, void *hip_stream);

/* out = -G*(P(F) - P-bar) (float64 device array of 9 x N), the right-hand side of
 * eq. (20) at the current F for the stress target Pbar (host, 9 values; only the
 * stress-controlled components are used).  Also refreshes P and the tangent state. */
int ghom_residual(ghom_ctx *ctx, const double Pbar[9], double *out_dev);

/* ---- kernel choices ----------------------------------------------------------------- */

/* Keys of ghom_set_option / ghom_get_option. */
enum {
  GHOM_OPT_XPROJ_F64 = 1,  /* x-pass (transform along x + projection) variant, float64    */
  GHOM_OPT_XPROJ_F32 = 2,  /* the same for the float32 transforms of GHOM_FP32_SPLIT      */
  GHOM_OPT_ZSLABS = 3,     /* number of kz slabs the y and x passes are run in (>= 1)     */
  GHOM_OPT_GRAPHS = 4,     /* 1: CG iterations are captured once into HIP graphs and
                              replayed (not while profiling is on); 0: launched one by one */
  GHOM_OPT_CHECKPOINTS = 5, /* 1: with the viscoelastic law, keep every accepted increment's
                              converged F and starting internal variables on the device
                              ((9 + 12) x N float64 each), as ghom_adjoint_grad_scale needs;
                              0: keep none (and drop those kept) */
  GHOM_OPT_STREAM_NT = 6,  /* 1: the transform passes load and store fields and spectra with
                              the nontemporal hint (no reuse expected in the last-level cache);
                              0: ordinary cached accesses.  Set at creation to 1 when one CG
                              iteration of all problems together touches more than 256 MB.
                              Passes along transform lines of length >= 128 always stream.
                              Results are the same either way. */
  GHOM_OPT_ROTATION_GAUGE = 7, /* 1 (default): the rotation gauge of full stress control (see
                              ghom_set_control); 0: the mask exactly as set.  Takes effect at
                              the next solve. */
  GHOM_OPT_YPASS_F64 = 8,  /* y-pass (transform along y) variant, float64                   */
  GHOM_OPT_YPASS_F32 = 9,  /* the same for the float32 transforms of GHOM_FP32_SPLIT         */
  GHOM_OPT_PROFILE_EVERY = 10 /* k >= 1 (default 1): with profiling on (ghom_set_profiling),
                              bracket only every k-th launch of each timed kernel name with
                              events; each bracketed launch costs a few microseconds of idle
                              GPU.  Setting it restarts the count. */
};

/* Selects a kernel variant.  For the x-pass keys: 0 = pick the fastest variant by timing
 * each on this GPU and grid (done by ghom_create; setting 0 re-times), 1 = "rows" (one
 * thread transforms the three components of a tensor row in turn), 2 = "groups" (three
 * thread groups, one per component, meeting in LDS), 3 = "rows" compiled for at least two
 * wavefronts per SIMD (fewer registers per thread), 4 = "rows" on the three-stage radix
 * schedule n = 8 x A1 x 8 (x lengths 128, 256, 512 only: 8 values per thread instead of
 * the two-stage split's B).  For the y-pass keys: 0 = pick by timing, 1 = "wide" (columns per
 * workgroup widened to 256-byte segments on lines >= 256), 2 = "narrow" (the plain column
 * count; only where it differs from "wide"), 3 = three-stage radix schedule (y lengths 128,
 * 256, 512).  A variant that does not exist for the grid returns GHOM_EINVAL.  All compute the
 * same operator.
 *
 * Tuning at creation is cached for the process, keyed by GPU architecture, pass, precision,
 * grid, problem count and streaming build, so a second context of the same shape reuses the
 * choice; with the environment variable GHOM_TUNE_CACHE naming a file, the cache is read from
 * that file and every new choice is appended to it.  Setting 0 always re-times. */
int ghom_set_option(ghom_ctx *ctx, int key, int value);

/* The kernel schedule the context runs, as text: grid, and per precision in use the x-pass
 * and y-pass variants with their radix splits ("16x16": 16 threads per line holding 16
 * values; "8x4x8": three stages, 32 threads holding 8) and whether the autotuner picked them.
 * Up to cap bytes (including the terminating zero) go to out (host; nullable).  Returns the
 * text's length, or GHOM_EINVAL. */
int ghom_get_schedule(ghom_ctx *ctx, char *out, int cap);

/* GHOM_OPT_ZSLABS: the y-forward, x (projection) and y-inverse passes are run slab by slab
 * over ranges of kz planes, so that a slab's intermediate spectrum can stay in the GPU's
 * last-level cache between the three passes (1 = one launch per pass). */

/* Reads the current value of an option (for the x-pass keys: the variant in use, 1, 2 or
 * 3, once tuned). */
int ghom_get_option(ghom_ctx *ctx, int key, int *value);

/* ---- measurement ------------------------------------------------------------------ */

/* Enables (1) or disables (0) HIP-event timing of every kernel launch of the context. */
int ghom_set_profiling(ghom_ctx *ctx, int on);

/* Restricts the timing to launches whose record name is exactly `name` (host string,
 * copied; NULL or "" times every launch again).  Each timed launch is bracketed by two
 * events on the context's stream, which costs a few microseconds per launch. */
int ghom_set_profiling_filter(ghom_ctx *ctx, const char *name);

/* Kernel timing records: number of distinct kernel names seen since profiling started. */
int ghom_profile_count(ghom_ctx *ctx);

/* Name, launch count and total milliseconds of record i (0 <= i < ghom_profile_count).
 * name_out receives at most name_cap bytes including the terminating zero.  Waits for
 * the context's stream. */
int ghom_profile_get(ghom_ctx *ctx, int i, char *name_out, int name_cap, int *launches,
                     double *total_ms);

/* Per-launch times of record i in milliseconds, in launch order: the first min(cap, count)
 * go to ms_out (host; NULL when cap is 0).  Returns the record's launch count, or a negative
 * status.  Launches that found nothing to do (CG iterations queued after a solve stopped,
 * which exit at once) are among them; a caller that wants the time of the launches that did
 * work separates them by their duration. */
int ghom_profile_samples(ghom_ctx *ctx, int i, float *ms_out, int cap);

/* Clears the timing records. */
int ghom_profile_reset(ghom_ctx *ctx);

/* ---- batches of independent problems ------------------------------------------------ */

/* Many cells and load cases advanced together (e.g. a set of RVEs under several load
 * paths).  Problems with the same grid and material law share every launch: each pass of
 * the method is one kernel launch per such group, whatever the number of problems. */
typedef struct ghom_batch ghom_batch;

enum { GHOM_MATERIAL_NEOHOOKEAN = 1, GHOM_MATERIAL_SVK = 2 };

/* One problem of a batch (host pointers, read by ghom_batch_create only).  The cell is the
 * unit cube.  kind selects the material law of ghom_set_material_neohookean (mu, lambda:
 * nphase values each) or ghom_set_material_svk (C: nphase x 81 values); phase has nx*ny*nz
 * entries; mask and target (nsteps x 9) as in ghom_set_control / ghom_set_history. */
typedef struct {
  int nx, ny, nz;
  int kind;
  const uint16_t *phase;
  int nphase;
  const double *mu, *lambda;
  const double *C;
  uint8_t mask[9];
  int nsteps;
  const double *target;
} ghom_problem;

/* Creates a batch of nprob problems (1..65535) in one precision on one device; all device
 * memory is allocated here.  hip_stream as in ghom_create. */
int ghom_batch_create(ghom_batch **out, const ghom_problem *probs, int nprob, int precision, int device,
                      void *hip_stream);

/* Releases the batch (NULL is ignored). */
void ghom_batch_destroy(ghom_batch *b);

/* Message of the last failed call on b. */
const char *ghom_batch_last_error(const ghom_batch *b);

/* Stopping rules shared by every problem (see ghom_set_tolerances). */
int ghom_batch_set_tolerances(ghom_batch *b, double newton_tol, double cg_tol, double cg_forcing,
                              int max_newton, int max_cg);

/* Advances every problem whose history is not exhausted by one increment.  info (nullable,
 * host) receives nprob records; problems not advanced have status GHOM_ESTATE.  Returns
 * GHOM_OK if every advanced problem converged, else the first failing problem's status
 * (the others are still advanced). */
int ghom_batch_step(ghom_batch *b, ghom_step_info *info);

/* <F> and <P> of problem iprob (host, 9 values each). */
int ghom_batch_get_averages(ghom_batch *b, int iprob, double Fbar[9], double Pbar[9]);

/* Field of problem iprob to host memory (as ghom_get_field). */
int ghom_batch_get_field(ghom_batch *b, int iprob, int which, double *host_out);

/* Kernel options of the batch (as ghom_set_option). */
int ghom_batch_set_option(ghom_batch *b, int key, int value);

/* Number of launch groups (distinct grid and material law) of the batch. */
int ghom_batch_num_classes(ghom_batch *b);

/* The kernel schedule of launch group cls (0 <= cls < ghom_batch_num_classes), as
 * ghom_get_schedule. */
int ghom_batch_get_schedule(ghom_batch *b, int cls, char *out, int cap);

#ifdef __cplusplus
}
#endif

#endif /* GHOM_H */
