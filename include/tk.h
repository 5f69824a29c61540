/*
 * tk.h -- C ABI of the MI355X Teukolsky m-mode time stepper.
 *
 * The library advances the complex fields (Phi, Pi) of one or many
 * azimuthal m-modes of the Teukolsky master equation (Eq. (1) of McKennon,
 * Forrester & Khanna, "High Accuracy Gravitational Waveforms from Black Hole
 * Binary Inspirals Using OpenCL", decomposed by their Eq. (2)) on 2+1D
 * (r*, theta) grids, with the two-step Lax-Wendroff scheme of Eqs. (3)-(4),
 * the angular and radial boundary conditions of Section 2.2, a smeared
 * Gaussian point-particle source (Section 2.3, item 1) and waveform sampling
 * (Section 5).  All stepping runs in HIP kernels on the device.
 *
 * Conventions
 *  - Units G = c = 1; M is the black hole mass, a its spin (|a| < M), s the
 *    spin weight (-2 <= s <= 2), m the azimuthal number.
 *  - Grid: r*_i = rstar_min + i h, h = (rstar_max - rstar_min)/(n_r - 1),
 *    i = 0 .. n_r-1;  theta_j = j pi/(n_theta - 1), j = 0 .. n_theta-1
 *    (poles included).
 *  - Host field arrays are row-major [theta_j][r*_i][re, im] (r* fastest,
 *    complex interleaved), n_theta * n_r * 2 doubles, caller-owned.
 *  - Device memory: the library allocates none for the fields.  The caller
 *    queries tk_workspace_bytes, allocates that much device memory (for
 *    instance a torch tensor) and binds it with tk_bind_workspace; it stays
 *    caller-owned and must outlive the context.  The autotuner's save area
 *    (tk_autotune_bytes) is caller-owned in the same way.  The library owns
 *    only small host structures, its timing events and captured graphs.
 *  - Every entry point returns a tk_status; on error the context is left
 *    unchanged and tk_last_error(ctx) describes the failure.  No C++
 *    exception crosses the ABI.
 *  - Work is enqueued on the HIP stream given to tk_init_grid.  Entry points
 *    that return host data (tk_get_fields, tk_extract) synchronise that
 *    stream first.  A context must not be used from two threads at once.
 */
#ifndef TK_H
#define TK_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TK_ABI_VERSION 5

typedef struct tk_ctx tk_ctx;

typedef enum {
    TK_OK = 0,
    TK_E_INVALID = 1,   /* bad argument or description; nothing changed     */
    TK_E_NOMEM = 2,     /* workspace too small / host allocation failed     */
    TK_E_DEVICE = 3,    /* a HIP call failed (message in tk_last_error)     */
    TK_E_STATE = 4,     /* call not allowed now (e.g. no workspace bound,   */
                        /* waveform ring overrun)                           */
    TK_E_UNSTABLE = 5,  /* dt above the scheme's stability bound            */
    TK_E_NONFINITE = 6  /* extracted samples contain NaN or Inf             */
} tk_status;

typedef enum {
    TK_FP64 = 0,      /* FP64 storage and arithmetic (the oracle-equivalent path) */
    TK_FP32_COMP = 1  /* FP32 storage and stencil arithmetic, compensated time
                         accumulation (bf16 compensation term per value), FP64
                         source injection                                    */
} tk_precision;

enum {
    TK_FLAG_FORCE_DT = 1 /* accept a dt above the stability bound */
};

/* One instance = one (a, s, m) mode on one grid.
 * Eqs. (2)-(4); the pole conditions (Section 2.2) follow from the parity of
 * m + s (a spin-weighted mode behaves like sin^{|m+s|} there; for the
 * paper's s = -2 this is the parity of |m|). */
typedef struct {
    double M, a;
    int s, m;
    int n_r, n_theta;     /* >= 5 each */
    double rstar_min, rstar_max;
    double dt;            /* time step (M) */
    double rstar_obs;     /* waveform column: node floor((rstar_obs - rstar_min)/h + 1/2) */
    int extract_every;    /* steps between waveform samples; 0 = no sampling  */
    int wave_capacity;    /* device ring size in samples (0 -> 4096)          */
    int flags;            /* TK_FLAG_* */
    /* Hyperboloidal outer layer (Section 2.3, item 2); 0 = none.  Otherwise
     * the nodes rho_i = rstar_min + i h are grid positions: r* = rho up to
     * rho = layer_start = R, and beyond it r* = rho / Omega(rho) with
     * Omega = 1 - ((rho - R) / (rstar_max - R))^4, so the last node
     * (rho = rstar_max) is future null infinity.  There the time is
     * tau = t - h(r*) with h' = H = 1 - d rho / d r* (tau = t below R), and
     * the second field is Pi~ = Pi / (1 - H b) (Pi below R): tk_set_fields
     * and tk_get_fields exchange (Phi, Pi~).  The last node takes the linear
     * extrapolation of the two nodes before it (no characteristic enters
     * there), so rstar_obs = rstar_max samples the waveform at null
     * infinity.  Requires s = -2 (whose Phi has a finite limit there),
     * max(0, rstar_min) < R, R + 2h <= rstar_max, and a particle source
     * confined to rho < R.  See tk_kernel for the kernels that step a
     * context with a layered instance. */
    double layer_start;
} tk_instance_desc;

typedef enum {
    TK_SRC_NONE = 0,
    TK_SRC_CIRCULAR_GAUSSIAN = 1,
    TK_SRC_CIRCULAR_STEP_DELTA = 2,
    TK_SRC_CIRCULAR_LINEAR_DELTA = 3
} tk_source_kind;

/* Smeared point particle (Section 2.3, item 1): the Pi equation gets
 *   F = amplitude * exp(-i m (Omega (t + t0) + phase0)) * g_r(r* - r*(r0)) * g_th(theta - pi/2)
 * with g(xi) = exp(-xi^2/(2 sigma^2)) / (sigma sqrt(2 pi)) for
 * |xi| <= window_sigmas * sigma and 0 beyond; sigma_r = sigma_r_cells * h,
 * sigma_th = sigma_th_cells * dtheta; Omega = sqrt(M)/(r0^{3/2} + a sqrt(M))
 * (prograde circular equatorial orbit).  Evaluated in FP64 in every
 * precision mode, at t^n in the first Lax-Wendroff step and t^n + dt/2 in
 * the second.
 *
 * Discrete-delta forms (Section 2.3, item 1: the finite-difference
 * derivative of a step function laid on the grid) replace g_r and g_th by
 * grid functions d(x - x_p) of unit sum times the spacing D (D = h in r*,
 * where nodes and half nodes each form a grid of spacing h; D = dtheta in
 * theta); sigma_*_cells and window_sigmas are then ignored:
 *   TK_SRC_CIRCULAR_STEP_DELTA: the centred difference of the sampled
 *     Heaviside step, d(x) = [H(x + D - x_p) - H(x - D - x_p)] / (2D) with
 *     H(0) = 1/2: 1/(2D) on the two grid points around x_p, or 1/(4D),
 *     1/(2D), 1/(4D) when x_p is on a grid point (within 1e-9 D, so that a
 *     particle on the equator sits on the row theta = pi/2 of an odd
 *     N_theta grid whatever the rounding of j dtheta);
 *   TK_SRC_CIRCULAR_LINEAR_DELTA: the difference of the step that rises
 *     linearly over one cell, d(x) = max(0, 1 - |x - x_p|/D) / D, exact on
 *     constants and linear functions (zeroth and first moments). */
typedef struct {
    int kind;
    double r0, amplitude, phase0;
    double sigma_r_cells, sigma_th_cells, window_sigmas;
    double t0; /* time along the orbit at step 0: a segment of a long run
                  (Section 4's temporal decomposition) starts at t0 */
    double ramp; /* switch-on time T_on (M; 0 = the full source from step
                    0): F is multiplied by s(t / T_on), t = n dt the time
                    since step 0 and s the smooth step
                    e^{-1/x} / (e^{-1/x} + e^{-1/(1-x)}) on 0 < x < 1 (0
                    below, 1 above), every derivative of which vanishes at
                    both ends, so that a run started from zero fields leaves
                    no persistent junk (Section 4's known techniques for the
                    junk burst of each segment) */
} tk_source_desc;

/* Kernel choice and launch shape (the only per-architecture tuning the
 * paper reports is the work-group size, Section 4). */
typedef enum {
    TK_KERNEL_AUTO = 0,     /* FUSED2 with rows_per_tile 0, else FUSED (FP32: the
                               fused forms only) */
    TK_KERNEL_TWO_PASS = 1, /* half-step array through HBM, one thread per point */
    TK_KERNEL_FUSED = 2,    /* both stages in one pass, theta-marching columns   */
    TK_KERNEL_FUSED2 = 3,   /* two time steps per pass over column strips (whole,
                               or chunks of rows_per_tile rows): u^n read and
                               u^{n+2} written once, u^{n+1} kept on chip (an
                               odd step count ends with one FUSED step);
                               results are bitwise those of FUSED */
    TK_KERNEL_TILED = 4     /* one step on tiles of rows_per_tile (4 or 8) rows
                               by 62 columns, one block of four waves per tile
                               with its rows staged in LDS: for grids too small
                               to give the marching kernels enough waves;
                               results are bitwise those of FUSED */
} tk_kernel;
/* A context with a hyperboloidal layer (tk_instance_desc.layer_start):
 * AUTO, FUSED2 and FUSED march whole instances as for plain ones, in a form
 * that takes the layer's coefficients beyond rho = R and extrapolates the
 * null-infinity column inside the pass (one u^n row in flight:
 * prefetch_rows is ignored); FUSED2 is again bitwise FUSED.  In
 * TK_FP32_COMP the layer's coefficients are in the compensated form's FP32
 * arithmetic and the null-infinity column is formed in double from the
 * stored pairs.  With rows_per_tile 0 the strips that reach a layer run in
 * chunks of 32 rows, the others whole.  TK_FP64 only, TWO_PASS: the layer's
 * half-step and full-step passes over whole instances (rows_per_tile: rows
 * per chunk, 0 = 16; the same results as FUSED up to rounding order).  TILED
 * is refused with TK_E_INVALID. */

enum {
    TK_TUNE_NT_STORES = 1 /* fused kernel: non-temporal stores of u^{n+1} */
};

typedef struct {
    int kernel;        /* tk_kernel */
    int rows_per_tile; /* fused kernels: theta rows per work item (0 = all;
                          FUSED2: 0 or >= 4, its chunks recompute the u^{n+1}
                          rows of a two-row halo; TILED: 4 or 8)              */
    int graph_steps;   /* steps per captured HIP graph (0 = no graphs)        */
    int prefetch_rows; /* fused kernel: u^n rows in flight per wave, 1 or 3 (0 = 3) */
    int flags;         /* TK_TUNE_* */
    int waves_per_simd;/* fused kernel: forced occupancy; must be 0 (the
                          compiler's register budget).  Budgets for 3 or 4
                          waves per SIMD spilled registers and never ran
                          faster, so they are not compiled: other values give
                          TK_E_INVALID */
} tk_tuning;

/* Set up the grids of n_inst instances on the host: the vertex-centred
 * (r*, theta) grid of Section 2.2 with the m-mode of Eq. (2) on each, the
 * tortoise inversion r(r*), and the radial and angular factors of the
 * first-order system that Eqs. (3)-(4) step (Eq. (1) divided by its Psi_tt
 * coefficient), plus the work decomposition.  No device memory is touched.
 * inst: n_inst host descriptions (copied; caller-owned).  hip_stream is a
 * hipStream_t; NULL is the legacy default stream, which cannot be captured,
 * so a context on it refuses graph_steps > 0.  Returns TK_E_UNSTABLE if some
 * instance's dt exceeds the stability bound of the scheme with its angular
 * terms (unless TK_FLAG_FORCE_DT), TK_E_INVALID for an invalid description
 * (the message names the instance).  On success *out owns the context. */
tk_status tk_init_grid(const tk_instance_desc *inst, int n_inst, tk_precision prec, void *hip_stream,
                       tk_ctx **out);

/* Bytes of device workspace the context needs (fields double-buffered,
 * tables, waveform rings). */
tk_status tk_workspace_bytes(const tk_ctx *ctx, size_t *bytes);

/* Bind caller-owned device memory of at least tk_workspace_bytes bytes
 * (256-byte aligned).  Uploads the tables and zeroes the fields and the
 * step counter.  May be called once per context. */
tk_status tk_bind_workspace(tk_ctx *ctx, void *dev_ptr, size_t bytes);

/* Copy host fields of instance inst into the current state (synchronous).
 * phi, pi: [n_theta][n_r][2] doubles.  Does not change the step counter. */
tk_status tk_set_fields(tk_ctx *ctx, int inst, const double *phi, const double *pi);

/* Copy the current state of instance inst to host arrays (synchronises). */
tk_status tk_get_fields(tk_ctx *ctx, int inst, double *phi, double *pi);

/* Set (or with kind = TK_SRC_NONE, remove) the particle source of inst. */
tk_status tk_set_source(tk_ctx *ctx, int inst, const tk_source_desc *src);

/* Advance every instance by n_steps full Lax-Wendroff steps (Eqs. (3)-(4)
 * with the Section 2.2 boundary conditions), asynchronously on the stream.
 * The state alternates between two buffers, one flip per kernel launch; the
 * context tracks which one is current.  With graph_steps = G > 0 (tuning)
 * the steps go as replays of one captured HIP graph of G steps, the
 * remainder as direct launches; TK_E_STATE if G > 0 on the NULL stream. */
tk_status tk_step(tk_ctx *ctx, long n_steps);

/* Do ahead of time the host-side work a later tk_step(n_steps) would do
 * first under the current tuning: upload the work list and, if
 * graph_steps = G > 0 and n_steps >= G, capture and instantiate the graph of
 * G steps.  Advances nothing.  Not for use during stream capture. */
tk_status tk_prepare(tk_ctx *ctx, long n_steps);

/* Launch counters of a context since tk_init_grid: graphs captured and
 * instantiated, graph replays, and direct (eager) kernel launches issued by
 * tk_step (autotuning is not counted). */
typedef struct {
    long graphs_instantiated;
    long graph_launches;
    long eager_launches;
} tk_counters;
tk_status tk_get_counters(const tk_ctx *ctx, tk_counters *out);

/* Waveform extraction (Section 5.1: the waveform read from Phi near the
 * outer boundary, at future null infinity with the layer of Section 2.3
 * item 2).  Copies the samples of inst taken since the last call, oldest
 * first, to out ([sample][theta][re, im] doubles, host memory, at most
 * max_samples samples, caller-owned) and drains them; *n_samples receives
 * the count.  Sample k holds Phi(t, r*_obs, theta_j) at
 * t = (k+1) extract_every dt after step counter 0.  Synchronises the
 * context's stream.  Returns TK_E_STATE if more samples than the ring holds
 * were produced since the last call (nothing is drained), TK_E_NONFINITE if
 * a copied sample is not finite (the samples are drained). */
tk_status tk_extract(tk_ctx *ctx, int inst, double *out, long max_samples, long *n_samples);

/* Step counter (steps taken since tk_bind_workspace or the last
 * tk_set_step); time of instance k is step * dt_k.  tk_set_step changes the
 * time index only: the current state is kept as it is (resume a
 * checkpoint with tk_set_step then tk_set_fields, in either order). */
tk_status tk_get_step(const tk_ctx *ctx, long *step);
tk_status tk_set_step(tk_ctx *ctx, long step);

/* Kernel variant / launch shape (TK_E_INVALID for unsupported values). */
tk_status tk_set_tuning(tk_ctx *ctx, const tk_tuning *t);
tk_status tk_get_tuning(const tk_ctx *ctx, tk_tuning *t);

/* Autotuner: time every compiled launch shape (kernel, u^n prefetch depth,
 * store kind; rows per tile 0, 32 and 16 for the two-step kernel, and, when
 * whole strips give fewer waves than two per SIMD of the device, the
 * smallest chunk of at least 4 rows that keeps the work list within that
 * many waves; 0, 64 and 16 for the one-step kernel, 8 and 4 for the tiled
 * kernel; a context with a hyperboloidal layer tries the shapes of its own
 * forms, see tk_kernel) on this context's own instances and keep the
 * fastest; graph_steps stays as it was.  Each candidate runs `warmup`
 * untimed and then `steps` timed steps (both rounded up to even), timed with
 * HIP events on the context's stream, in two passes over the candidates in
 * opposite orders (its faster time counts).  The state, the step counter and
 * the waveform rings are copied to save_area and restored afterwards, so the
 * simulation is left as it was found.  save_area: caller-owned device memory
 * of at least tk_autotune_bytes bytes, 256-byte aligned, free for the
 * duration of the call (the library allocates nothing).  Synchronous; not
 * for use during stream capture.  On success *best_ms_per_step and *n_tried
 * (each may be NULL) receive the winner's time per step and the number of
 * shapes timed.  TK_E_NOMEM if save_bytes is too small, TK_E_INVALID if
 * save_area is not aligned device memory. */
tk_status tk_autotune_bytes(const tk_ctx *ctx, size_t *bytes);
tk_status tk_autotune(tk_ctx *ctx, int warmup, int steps, void *save_area, size_t save_bytes,
                      double *best_ms_per_step, int *n_tried);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture elsewhere in the process, tight serving loops, harnesses that
 * forbid allocation): tk_autotune with its save area taken from a static
 * scratch array inside the library instead of from the caller.  The array
 * holds TK_AUTOTUNE_STATIC_MAX_BYTES (64 MiB) on each GPU the library runs
 * on, from the first call on that GPU until the process ends; its address on
 * the context's device is looked up on that first call.  A context whose
 * tk_autotune_bytes exceeds it gets TK_E_NOMEM (nothing changed; use
 * tk_autotune with a caller save area).  The call allocates no device memory
 * and frees none.  Every call on one GPU shares that GPU's array, whose
 * contents are overwritten before they are read; calls from one process are
 * serialised, and calls from different processes have arrays of their own,
 * so overlapping calls do not mix their saves, but they do time their
 * candidates against each other.  Arguments, results and the restored
 * simulation are those of tk_autotune. */
#define TK_AUTOTUNE_STATIC_MAX_BYTES ((size_t)64 << 20)
tk_status tk_autotune_static(tk_ctx *ctx, int warmup, int steps, double *best_ms_per_step, int *n_tried);

/* Wait for all work enqueued by the context. */
tk_status tk_synchronize(tk_ctx *ctx);

/* Release the context (never frees the caller's workspace). */
tk_status tk_destroy(tk_ctx *ctx);

/* Last error message of ctx (or of the last failed tk_init_grid if ctx is
 * NULL).  Valid until the next call on the same context. */
const char *tk_last_error(const tk_ctx *ctx);

/* Largest stable dt of the scheme for one description (same rule as the
 * TK_E_UNSTABLE check); the description's own dt is not used. */
tk_status tk_stable_dt(const tk_instance_desc *inst, double *dt_max);

/* Richardson extrapolation of second-order results (Section 2.3, item 3)
 * and its error estimate from two extrapolants (Section 5.1, footnote).
 * w1, w2, w3: n complex values each ([k][re, im], host memory, caller-owned)
 * of the same quantity computed with the grid spacings and time step scaled
 * by 1, 1/2, 1/4 (for waveforms: the same sample times and observer).  With
 * q = 2^order:
 *   R12 = (q w2 - w1) / (q - 1),  R23 = (q w3 - w2) / (q - 1);
 * extrap[k] = R23[k]; err[k] = |R23[k] - R12[k]| / |R23[k]| (the absolute
 * difference where R23[k] = 0).  extrap and err may be NULL.  A host
 * computation, O(n); TK_E_INVALID for n < 0, order < 1 or a NULL input, and
 * TK_E_NONFINITE if an input value is not finite. */
tk_status tk_richardson(const double *w1, const double *w2, const double *w3, long n, int order, double *extrap,
                        double *err);

int tk_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* TK_H */
