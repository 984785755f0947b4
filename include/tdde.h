/*
 * tdde.h -- C ABI of the MI355X (gfx950) Crank-Nicolson / BiCGSTAB time step for the
 * time-dependent Dirac equation in a spherical-spinor x B-spline basis.
 *
 * Method (arXiv 2512.21697, "GaDE"):
 *   - Hamiltonian, eq. fullH:  H(t) = H0 + sum_m coef_m f_m(t) (K^a A_m K^b) (x) R_m
 *     H0 (and the overlap S) are block diagonal over angular channels j and are polynomials
 *     in the channel's kappa; A_m are sparse angular couplings, R_m banded radial matrices
 *     (2x2 grid of bands over the large/small spinor components, Sec. 2.2).
 *   - time step, eq. solPsi with the midpoint rule of Sec. 2.4:
 *       (S + i dt/2 H(t_n + dt/2)) psi_{n+1} = (S - i dt/2 H(t_n + dt/2)) psi_n
 *   - linear solve by BiCGSTAB (Sec. 2.4, Sec. 3.3), optionally right-preconditioned with
 *     the LU factors of the block-diagonal M = S + i dt/2 H0 (eq. matrixM).
 *   - time functions f_m(t): sin^2-envelope pulses (eq. ndpPot, dipole limit) and their
 *     trigonometric factorisation (eq. bdpA).
 *
 * Conventions
 *   - Complex numbers are interleaved (re, im) pairs: tdde_c128 / float pairs for c64.
 *   - State vectors are device arrays laid out [batch][nang][2][nr] (instance, channel,
 *     component s = 0 large / 1 small, radial index), contiguous, complex128 unless a
 *     function says complex64. The caller owns them; the library never frees them and
 *     never keeps a pointer past the call.
 *   - Band arrays are host arrays [..][2][2][2*half_band+1][nr]: band[s][s'][d+hb][i]
 *     multiplies x[s'][i+d] into y[s][i]; entries whose column falls outside [0, nr) must be 0.
 *   - All work is enqueued on the stream given to tdde_create (a hipStream_t passed as void*,
 *     NULL = default stream). Functions that return host statistics synchronise that stream.
 *   - Every function returns a tdde_status; nothing throws across the ABI. On error the
 *     context stays usable and tdde_last_error() describes the failure.
 *   - Memory: tdde_assemble allocates every device buffer the context needs (operator copy,
 *     Krylov workspace, reduction scratch); tdde_set_dt the preconditioner factors on its first
 *     call; tdde_set_field_table its table when it grows. tdde_set_pulses, tdde_set_field, tdde_apply, tdde_solve, tdde_solve_static,
 *     tdde_step, tdde_run_batched allocate nothing.
 */
#ifndef TDDE_H
#define TDDE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TDDE_OK = 0,
  TDDE_NOT_CONVERGED = 1, /* max_iter reached; x holds the last iterate, stats are filled      */
  TDDE_BREAKDOWN = 2,     /* repeated BiCGSTAB breakdown (rho or omega vanished after restart)  */
  TDDE_NONFINITE = 3,     /* NaN or Inf in the right-hand side, guess or iteration; the solve    */
                          /* stopped at the first reduction that saw it (x: the last iterate)    */
  TDDE_ERR_ARG = -1,      /* bad argument or shape; nothing was launched                        */
  TDDE_ERR_HIP = -2,      /* a HIP call failed; message in tdde_last_error                      */
  TDDE_ERR_NOMEM = -3,    /* device allocation failed in tdde_assemble                          */
  TDDE_ERR_STATE = -4     /* call order violated (e.g. solve before assemble / set_dt)          */
} tdde_status;

typedef struct { double re, im; } tdde_c128;

typedef struct tdde_ctx tdde_ctx; /* opaque; use one context per stream / host thread */

typedef struct {
  int32_t nr;        /* radial functions per component (B-spline count after boundary trim) */
  int32_t nang;      /* angular channels (kappa, mu)                                         */
  int32_t half_band; /* radial half-bandwidth hb; must be 6 (order-7 B-splines, Sec. 2.2)     */
  int32_t batch;     /* independent instances sharing the operator (different fields)        */
  int32_t n_fields;  /* time functions per instance                                          */
} tdde_dims;

/* Operator description (host pointers, copied by tdde_assemble; the caller keeps ownership).
 * Restates eq. fullH:  H0 block j = sum_n kappa_j^n h_poly[n] (+ h_chan[j]),
 *                      S block j = sum_n kappa_j^n s_poly[n] (identity when n_s = 0),
 *                      V_m = (K^a A_m K^b) (x) R_m with K = diag(kappa). */
typedef struct {
  const double* kappa;      /* [nang]                                                        */
  int32_t n_h;              /* number of kappa-polynomial H0 terms (0..4)                    */
  const double* h_poly;     /* [n_h][2][2][2hb+1][nr] real, or NULL when n_h == 0            */
  const double* h_chan;     /* [nang][2][2][2hb+1][nr] complex (re, im pairs) or NULL        */
  int32_t n_s;              /* number of kappa-polynomial S terms (0 = identity, 1..3)       */
  const double* s_poly;     /* [n_s][2][2][2hb+1][nr] real, or NULL                          */
  int32_t n_terms;          /* coupling terms                                                */
  const int32_t* a_rowptr;  /* [n_terms][nang+1] CSR row pointers, offsets into a_col/a_val  */
                            /* counted from the start of each term's own slice               */
  const int64_t* a_off;     /* [n_terms+1] start of each term's slice in a_col / a_val       */
  const int32_t* a_col;     /* concatenated CSR column indices (channels)                    */
  const double* a_val;      /* concatenated CSR values (real)                                */
  const double* r_band;     /* [n_terms][2][2][2hb+1][nr] real radial bands                  */
  const int32_t* kpow;      /* [n_terms][2] exponents (a, b) of K^a A_m K^b                  */
  const double* coef;       /* [n_terms][2] complex prefactor coef_m                         */
  const int32_t* field;     /* [n_terms] index of the time function f multiplying term m     */
} tdde_operator_desc;

/* One time function: f(t) = amp * env(t) * sin(omega t + phase) for 0 < t < T, else 0;
 * env = sin^2(pi t / T) when envelope != 0, else 1 (eq. ndpPot in the dipole limit; a cosine
 * factor of eq. bdpA is phase = pi/2). */
typedef struct {
  double amp, T, omega, phase;
  int32_t envelope, pad_;
} tdde_pulse;

enum { TDDE_GUESS_ZERO = 0, TDDE_GUESS_PREV = 1, TDDE_GUESS_GIVEN = 2 };
enum { TDDE_PREC_FP64 = 0, TDDE_PREC_MIXED = 1 };

typedef struct {
  double tol;          /* stop when ||b - A x||_2 <= tol ||b||_2 (recursive, then true residual) */
  int32_t max_iter;    /* BiCGSTAB iterations per solve (per inner solve in mixed mode)           */
  int32_t guess;       /* TDDE_GUESS_*                                                            */
  int32_t precond;     /* 0 = none, 1 = block-diagonal LU of M = S + i dt/2 H0 (eq. matrixM)      */
  int32_t precision;   /* TDDE_PREC_FP64, or TDDE_PREC_MIXED: FP64 iterative refinement around an */
                       /* FP32 (complex64) BiCGSTAB; residuals, dots and corrections in FP64       */
  double inner_tol;    /* mixed only: relative tolerance of each FP32 inner solve (e.g. 1e-5)     */
  int32_t max_outer;   /* mixed only: refinement steps                                            */
  int32_t pad_;
} tdde_solve_opts;

/* Per-instance statistics of one solve / step. */
typedef struct {
  int32_t status;       /* tdde_status of this instance; TDDE_ERR_HIP if the launch's grid     */
                        /* barrier timed out before the step finished (step not completed)     */
  int32_t iters;        /* BiCGSTAB iterations (a converged half iteration counts as one)     */
  int32_t matvecs;      /* operator applications, residual checks included (a residual check   */
                        /* that also forms the next step's right-hand side counts once)        */
  int32_t restarts;     /* breakdown or failed true-residual restarts                          */
  int32_t outer_iters;  /* refinement steps (mixed precision), else 0                          */
  int32_t precs;        /* preconditioner solves (block LU of eq. matrixM)                     */
  double rel_res;       /* recursive residual at exit / ||b||                                  */
  double true_rel_res;  /* ||b - A x|| / ||b|| at exit                                         */
} tdde_solve_stats;

/* Create a context for the given sizes on `hip_stream` (hipStream_t or NULL). Allocates nothing
 * on the device (it resolves, once per device, the address of the static scratch array behind
 * tdde_solve_static). Errors: TDDE_ERR_ARG for nonpositive sizes, half_band != 6 or n_fields > 16.
 * Paper: the per-rank set-up before the time loop (Sec. 3.1, the implementation steps). */
tdde_status tdde_create(const tdde_dims* dims, void* hip_stream, tdde_ctx** out);

/* Copy the operator to the device (FP64 and FP32 copies) and allocate every workspace buffer.
 * May be called once per context. Errors: TDDE_ERR_ARG (inconsistent CSR, kappa exponents with
 * zero kappa, field index out of range), TDDE_ERR_NOMEM, TDDE_ERR_HIP.
 * Paper: the operator of eq. fullH (h and g sub-matrices, the angular coupling H^theta) copied to
 * the device once and memory allocated once before the time loop (Sec. 3.1, steps 2 and 5). */
tdde_status tdde_assemble(tdde_ctx* ctx, const tdde_operator_desc* desc);

/* Set the time step. Factors M = S + i dt/2 H0 per distinct channel block (banded LU without
 * pivoting, valid because the Hermitian part of M is the SPD overlap S) and uploads the
 * factors. Must follow tdde_assemble. Allocates the factor buffers on its first call.
 * Paper: the preconditioner of eq. matrixM, factored once at start-up (Sec. 2.4; Sec. 3.1 step 4). */
tdde_status tdde_set_dt(tdde_ctx* ctx, double dt);

/* Pulses of every instance: host array [batch][n_fields]. Used by tdde_step / tdde_run_batched,
 * which evaluate f at the midpoint time of each step on the device (this replaces a field table
 * set with tdde_set_field_table). Paper: the sin^2-envelope time functions of eq. ndpPot and
 * eq. bdpA, evaluated at the midpoint t + dt/2 of Sec. 2.4. */
tdde_status tdde_set_pulses(tdde_ctx* ctx, const tdde_pulse* pulses);

/* Field table: host array f[batch][n_rows][n_fields]; row n holds the time functions f_m at the
 * midpoint of step n (tdde_run_batched's step index, t = t0 + (n + 1/2) dt; tdde_step takes row 0).
 * Replaces the pulses for the steps that follow (tdde_set_pulses switches back), so the library is
 * not tied to one pulse family: the caller tabulates any f_alpha(t) of eq. bdpA. Allocates the
 * device copy on its first call and when the table grows. Errors: TDDE_ERR_ARG (n_rows < 1,
 * non-finite values), TDDE_ERR_NOMEM; tdde_run_batched returns TDDE_ERR_ARG, before any launch, when
 * a step it would run has no row. Paper: the scalar time functions of eq. fullH computed for each
 * step (Sec. 3.1 step 2a), here supplied by the caller. */
tdde_status tdde_set_field_table(tdde_ctx* ctx, const double* f, int32_t n_rows);

/* The pulses of tdde_set_pulses evaluated on the device at the midpoints of steps step0 .. step0+n-1
 * (t = t0 + (k + 1/2) dt, the times the time steps use, same arithmetic) into the host array
 * f[batch][n][n_fields]; synchronises the stream. Uses the right-hand-side workspace (do not overlap
 * with a step on another stream); batch * n * n_fields <= 2 * batch * nang * 2 * nr. Paper: the
 * sin^2-envelope time functions of eq. ndpPot / eq. bdpA. */
tdde_status tdde_eval_pulses(tdde_ctx* ctx, double t0, int32_t step0, int32_t n, double* f);

/* Explicit field values f[batch][n_fields] (host) used by tdde_apply, tdde_solve and
 * tdde_solve_static. Paper: the scalar time functions f_alpha(t) that multiply the coupling terms
 * of eq. fullH (computing H(t) for a step, Sec. 3.1 step 2a). */
tdde_status tdde_set_field(tdde_ctx* ctx, const double* f);

/* y = a_s * S x + a_h * H x for every instance, with the fields of tdde_set_field.
 * x, y: device [batch][nang][2][nr] complex128, x != y. No synchronisation.
 * Paper: the product H x of eq. fullH (the SpMV of Sec. 3.3, here matrix-free). */
tdde_status tdde_apply(tdde_ctx* ctx, tdde_c128 a_s, tdde_c128 a_h, const void* x_dev, void* y_dev);

/* Same in complex64 with the FP32 operator copy (FP32 accumulation): the inner apply of the mixed
 * precision solve (an addition to the paper's FP64 method, Sec. 4 reports FP64 complex only). */
tdde_status tdde_apply_c64(tdde_ctx* ctx, tdde_c128 a_s, tdde_c128 a_h, const void* x_dev, void* y_dev);

/* Apply the block preconditioner: z = M^-1 v (complex128, device, [batch][nang][2][nr]).
 * Needs tdde_set_dt. Paper: the LU solve with the factors of eq. matrixM (Sec. 2.4). */
tdde_status tdde_precond_apply(tdde_ctx* ctx, const void* v_dev, void* z_dev);

/* Solve (S + i dt/2 H) x = b with the fields of tdde_set_field. b, x: device complex128
 * [batch][nang][2][nr]; x holds the initial guess on entry (opts->guess must be GIVEN or ZERO)
 * and the solution on exit. stats: host array [batch] or NULL (NULL = no synchronisation).
 * Returns TDDE_NOT_CONVERGED / TDDE_BREAKDOWN when any instance did not converge.
 * Paper: the BiCGSTAB solve of the Crank-Nicolson system eq. solPsi (Sec. 2.4, Sec. 3.1 step 2b). */
tdde_status tdde_solve(tdde_ctx* ctx, const void* b_dev, void* x_dev, const tdde_solve_opts* opts,
                       tdde_solve_stats* stats);

/* Size of the static device array behind tdde_solve_static (per GPU, held until the process ends). */
#define TDDE_STATIC_SCRATCH_BYTES (64ll << 20)

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): tdde_solve with the solve's scratch (the iterate and
 * eight Krylov vectors, a right-hand-side copy, reduction partials, grid-barrier words, counters
 * and the statistics) in a library-owned static device array of TDDE_STATIC_SCRATCH_BYTES per GPU
 * instead of the context's workspace; same kernels and results as tdde_solve. Calls no allocation
 * routine. Needs 10 * batch * nang * 2 * nr * 16 bytes plus about 240 KB; larger solves and mixed
 * precision return TDDE_ERR_ARG before any launch (the limit is about 417,000 complex unknowns
 * over all instances). Every call on one GPU uses the same array and finds the previous call's
 * contents there (the kernels clear what must start at zero): calls that overlap in time on one
 * GPU (several streams or host threads) race and give wrong results; serialise them. The context
 * must have been created with the device current. Arguments and errors as tdde_solve. */
tdde_status tdde_solve_static(tdde_ctx* ctx, const void* b_dev, void* x_dev, const tdde_solve_opts* opts,
                              tdde_solve_stats* stats);

/* One time step of every instance from time t: evaluates f_m(t + dt/2) from the pulses (or takes
 * row 0 of the field table), forms b = (S - i dt/2 H) psi, solves with BiCGSTAB from the chosen
 * guess, writes psi_{n+1} into psi. guess_dev: device complex128 guess when opts->guess == GIVEN,
 * else ignored (may be NULL). stats: host [batch] or NULL.
 * Paper: one step of the time loop, eq. solPsi with the midpoint rule (Sec. 2.4, Sec. 3.1 step 2). */
tdde_status tdde_step(tdde_ctx* ctx, void* psi_dev, double t, const void* guess_dev, const tdde_solve_opts* opts,
                      tdde_solve_stats* stats);

/* Advance every instance by up to n_chunk steps in one persistent launch. Instance b advances
 * from step index step0 while step < n_steps[b] (host array [batch]); time t = t0 + step * dt.
 * Paper: the time loop of Sec. 3.1 step 2 run fully on the device (Sec. 3.3), for a batch of
 * independent instances that share the operator (an addition to the paper: different fields).
 * guess_dev: device complex128 [batch][E] initial guess, required when opts->guess == GIVEN (then
 * n_chunk must be 1), else ignored. stats_dev: device array [n_chunk][batch] of tdde_solve_stats,
 * or NULL. No host synchronisation. */
tdde_status tdde_run_batched(tdde_ctx* ctx, void* psi_dev, double t0, int32_t step0, int32_t n_chunk,
                             const int32_t* n_steps, const void* guess_dev, const tdde_solve_opts* opts,
                             void* stats_dev);

/* Photoelectron energy spectrum, eq. dPdE: dP/dE = sum over channels (kappa, mu) of
 * |<psi_{kappa,mu,E}|Psi>|^2 with the field-free eigenstates of each channel's radial block (Sec. 2.3:
 * H0 v = E S v), found by diagonalisation before the run (the paper's pre-computed input, Sec. 3.1)
 * and passed in here: n_blk eigen-blocks (channels of one block share kappa, hence H0, S and the
 * eigenvectors: Sec. 2.2, the blocks depend on kappa only); blk_of[nang] the block of every channel;
 * per block n_lev[b] levels inside the energy window, ascending (levels: concatenated over blocks)
 * and edges[b][2] the nearest levels below and above the window; vecs [total levels][2][nr] the
 * real box-normalised eigenvectors (v^T S v = 1); grid[n_grid] ascending energies. A level stands
 * for the energy-normalised state times sqrt(dE_n), dE_n = (E_{n+1} - E_{n-1}) / 2, so the density
 * at E_n is |v_n^T S Psi_j|^2 / dE_n; each channel's density is interpolated linearly onto the grid
 * (zero outside its levels) and the channels are summed. Host arrays, copied; allocates the
 * spectrum buffers (once per context). Needs real kappa-polynomial blocks (no per-channel bands).
 * Errors: TDDE_ERR_ARG (indices, orders, sizes), TDDE_ERR_STATE (before assembly, or a second call). */
tdde_status tdde_spectrum_setup(tdde_ctx* ctx, int32_t n_blk, const int32_t* blk_of, const int32_t* n_lev,
                                const double* levels, const double* edges, const double* vecs, const double* grid,
                                int32_t n_grid);

/* dP/dE on the grid for every instance: psi_dev [batch][nang][2][nr] complex128, dpde_dev
 * [batch][n_grid] double (device). No synchronisation. Paper: eq. dPdE. */
tdde_status tdde_spectrum(tdde_ctx* ctx, const void* psi_dev, void* dpde_dev);

/* Spectral error of Sec. 4 (physical validation): err[b] = integral over the grid of
 * |P_b(E) - Q_b(E)|^2 dE (trapezoidal rule); p_dev, q_dev [batch][n_grid] double (device), err host
 * [batch]; synchronises the stream. */
tdde_status tdde_spectrum_error(tdde_ctx* ctx, const void* p_dev, const void* q_dev, double* err);

/* Release every device buffer of the context. Accepts NULL. */
tdde_status tdde_destroy(tdde_ctx* ctx);

/* Launch shape of the persistent kernel: at most wg_per_cu work-groups per compute unit (1..4;
 * 0 restores the default, 4), further capped by each kernel variant's occupancy. The GPU mapping
 * of the solver's kernels (Sec. 3.3) leaves the number of thread blocks open; this is the knob the
 * launch autotuner sweeps. Results agree between shapes up to the order of the grid-wide
 * reductions. Call after tdde_assemble. TDDE_ERR_ARG when wg_per_cu is out of range or the grid
 * would hold fewer work-groups than instances (nothing is changed then); TDDE_ERR_STATE before
 * assembly. */
tdde_status tdde_set_launch(tdde_ctx* ctx, int32_t wg_per_cu);

/* Graph mode (on != 0) for tdde_step / tdde_run_batched / tdde_solve: the launch sequence of a
 * persistent chunk (two fill kernels and the cooperative solver launch) is captured into a HIP graph
 * on the context's stream once per kernel variant and grid and replayed with each call's arguments
 * (the paper runs its time loop fully on the device, Sec. 3.3; a graph removes the per-chunk launch
 * work from the host). The context's stream must not be the legacy default stream. A runtime that
 * cannot capture the cooperative launch makes the call return TDDE_ERR_HIP with the HIP error text
 * (the context stays usable in direct mode). Off by default; phase marks use direct launches. */
tdde_status tdde_set_graph(tdde_ctx* ctx, int32_t on);

/* Launch-shape knob of the preconditioner's segmented triangular solves (eq. matrixM applied
 * through its LU factors): each channel's 2 nr rows are split into segments of at least min_rows rows
 * (one per thread, at most 256 per channel; default 24). Longer segments mean fewer boundary
 * matrices and longer sequential substitution chains; the autotuner times the choices. Takes effect
 * at the next tdde_set_dt (which refactors). TDDE_ERR_ARG when min_rows < 13 or > 4096. */
tdde_status tdde_set_prec_segment(tdde_ctx* ctx, int32_t min_rows);

/* Solver form of time steps with the previous-state guess in FP64 (tdde_step, tdde_run_batched with
 * guess TDDE_GUESS_PREV and precision TDDE_PREC_FP64): on = 0 (default) runs a call as one
 * persistent cooperative launch; on = 1 runs every window of the BiCGSTAB iteration (van der Vorst
 * 1992; the iteration of eq. solPsi, right preconditioner of eq. matrixM when enabled) as a kernel of
 * its own, each at the occupancy its registers allow, with the scalar recurrence in device memory
 * and every decision taken by the last work-group of the instance (deterministic sums). The same
 * iteration, convergence tests, restarts and statistics as the persistent form; iterates agree to the
 * solve tolerance (sums in another grouping). A call in this form returns when its steps are done:
 * the host enqueues one iteration's kernels at a time and reads the count of unfinished instances one
 * iteration behind (it cannot be captured into a graph). psi is the iterate itself. Other guess modes,
 * mixed precision and tdde_solve keep the persistent form. Allocates the control blocks, partials and
 * two ints of pinned host memory on the first call with on = 1. TDDE_ERR_STATE before tdde_assemble;
 * TDDE_ERR_ARG for on outside {0, 1}. */
tdde_status tdde_set_split(tdde_ctx* ctx, int32_t on);

/* Storage precision of the preconditioner's factors (eq. matrixM: the LU of M = S + i dt/2 H0 and its
 * segment coupling matrices) read by the kernel-per-window solver: 64 (default) or 32 bits. With 32
 * the factors are the FP64 factorisation rounded to FP32 (the copy the mixed-precision solver uses);
 * substitutions, vectors and every residual stay FP64, and convergence is still decided by the FP64
 * true residual, so only the preconditioner (already an approximation of A: it omits the coupling)
 * changes, by ~1e-7 relative. TDDE_ERR_ARG for other values. */
tdde_status tdde_set_prec_storage(tdde_ctx* ctx, int32_t bits);

/* Persistent-grid size actually used (work-groups) and the per-instance work-group count. */
tdde_status tdde_launch_info(tdde_ctx* ctx, int32_t* n_wg, int32_t* wg_per_instance);

/* Diagnostics (no passage of the paper: measurement support, Sec. 4 reports wall times per step):
 * record up to cap phase timestamps of work-group 0 in every later persistent launch
 * (value = (wall_clock64 << 8) | phase id; the device wall clock runs at 100 MHz on gfx950).
 * cap = 0 disables. tdde_debug_read_marks synchronises the stream and copies them to the host. */
tdde_status tdde_debug_phase_marks(tdde_ctx* ctx, int32_t cap);
tdde_status tdde_debug_read_marks(tdde_ctx* ctx, uint64_t* host, int32_t cap);

/* Diagnostics of the kernel-per-window form (tdde_set_split): record a pair of HIP events on the
 * context's stream around each of the next cap launches of its apply kernel v = A p^ (the operator
 * apply fused with <r^, v>), so that its launch durations are measured on the stream it runs on;
 * cap = 0 disables. tdde_debug_read_split_timing waits for the recorded events, writes the duration
 * of each recorded launch in milliseconds (launches in blocks that found no work included: they end
 * at once), returns their count in *n (at most cap_host) and starts a new recording. */
tdde_status tdde_debug_split_timing(tdde_ctx* ctx, int32_t cap);
tdde_status tdde_debug_read_split_timing(tdde_ctx* ctx, float* ms, int32_t cap_host, int32_t* n);

/* Test hook (no passage of the paper: it drives the breakdown branch of the iteration): shadow
 * residual r^ of the first BiCGSTAB cycle of every later tdde_solve / tdde_solve_static, a device
 * complex128 array [batch][nang][2][nr] that must stay valid while those calls run (NULL restores
 * r^ = r0). A shadow with <r^, r0> = 0 makes rho vanish at once, and the solve restarts with
 * r^ = r; steps (tdde_step, tdde_run_batched) always take r^ = r0. */
tdde_status tdde_debug_set_shadow(tdde_ctx* ctx, const void* shadow_dev);

/* Error reporting of the ABI (no passage of the paper): text of a status / of the context's last error. */
const char* tdde_status_string(tdde_status s);
const char* tdde_last_error(const tdde_ctx* ctx); /* NULL ctx: last create error */

#ifdef __cplusplus
}
#endif
#endif /* TDDE_H */
