/* af_mhd.h -- C ABI of the MI355X (gfx950) library for one SSP-RK3 stage of
 * the positivity-preserving Active Flux scheme for 2D ideal MHD with the
 * Godunov-Powell source term (Duan, Chandrashekar, Klingenberg,
 * arXiv 2506.04857).
 *
 * The method: Section 2 (cell-average and point-value updates), Section 3
 * (first-order LLF scheme, parametrized flux limiter, scaling limiter, shock
 * sensor), time integration by SSP-RK3 whose stages are convex combinations
 * of forward-Euler steps (Sections 2 and 3.1).
 *
 * Degrees of freedom on an nx x ny Cartesian grid with spacings dx, dy
 * (0-based; fig. 2d_af_dofs):
 *   A(i,j)  cell average of cell (i,j)
 *   X(k,j)  point value at (x_{k-1/2}, y_j)        left vertical face of cell k
 *   Y(i,l)  point value at (x_i, y_{l-1/2})        bottom horizontal face of cell i
 *   V(k,l)  point value at (x_{k-1/2}, y_{l-1/2})  lower-left vertex of cell (k,l)
 * A periodic direction holds n entries per point set, an outflow direction
 * n+1 (the boundary nodes on both sides).  Conservative variables in the
 * paper's order U = (rho, rho v1, rho v2, rho v3, B1, B2, B3, E).
 *
 * Memory: every array is FP64, structure of arrays, component-major, x
 * fastest, C-contiguous, in device memory of the current HIP device:
 *   cell  [8][ny ][nx ]
 *   xface [8][ny ][nxp]   nxp = nx (periodic x) or nx+1 (outflow x)
 *   yface [8][nyp][nx ]   nyp = ny (periodic y) or ny+1 (outflow y)
 *   vert  [8][nyp][nxp]
 * The caller owns all device memory (states and the workspace); the library
 * never allocates device memory.  Pointers must be 8-byte aligned.
 *
 * Asynchrony: af_mhd_dt, af_mhd_stage and af_mhd_step only enqueue work on
 * the context's stream and never synchronise; the time step lives in device
 * memory.  af_mhd_stats synchronises the stream.
 *
 * Errors: functions return an af_status; none aborts.  A context is not
 * thread-safe; several contexts may coexist.
 */
#ifndef AF_MHD_H
#define AF_MHD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  AF_OK = 0,
  AF_EINVAL = -1,          /* invalid argument: null/misaligned pointer, bad size, bad k */
  AF_EHIP = -2,            /* a HIP runtime call failed; see af_mhd_last_error */
  AF_EWORKSPACE = -3,      /* workspace smaller than af_mhd_workspace_bytes */
  AF_ENOTADMISSIBLE = -4   /* af_mhd_stats: some degree of freedom is outside G (rho<=0 or p<=0) */
} af_status;

enum { AF_BC_PERIODIC = 0, AF_BC_OUTFLOW = 1 };

typedef struct {
  int32_t nx, ny;           /* cells per direction, each >= 4 */
  double x0, x1, y0, y1;    /* domain; dx = (x1-x0)/nx, dy = (y1-y0)/ny */
  double gamma;             /* adiabatic index of the perfect gas EOS, > 1 (Section 1) */
  double cfl;               /* dt = cfl / max over all DoFs of (rho_1/dx + rho_2/dy), in (0,1] */
  double kappa;             /* shock-sensor strength (Section 3.4), >= 0; 0 disables the sensor */
  int32_t bc_x, bc_y;       /* AF_BC_PERIODIC or AF_BC_OUTFLOW per direction */
  uint32_t flags;           /* AF_FLAG_* bits below; other bits are rejected */
} af_mhd_params;

/* FP32-bulk stage: fluxes, wave speeds, the flux-vector-splitting and LLF
 * sums, the shock sensor and the source sums in FP32; storage, pressure
 * recovery (the rho E - |m|^2/2 - rho |B|^2/2 cancellation), the centre
 * value, every stage accumulation U + dt RHS, every positivity-limiter
 * decision and the limiter's root solves stay FP64.  Results then differ
 * from the FP64 stage at the FP32 rounding level (about 1e-7 relative per
 * stage); the limiters still guarantee rho, p >= the paper's bounds. */
#define AF_FLAG_FP32_BULK 1u

/* Record HIP events on the context's stream around every kernel launch so
 * that af_mhd_kernel_times can report per-kernel device time.  Costs one
 * event record per launch boundary; off by default. */
#define AF_FLAG_KERNEL_TIMING 4u

/* Time-step reduction fused into the epilogue of a step's last stage:
 * af_mhd_step leaves, per workgroup of its stage-2 kernels, the maximum of
 * rho_1/dx + rho_2/dy over the values it stores, and the next af_mhd_step
 * on the same state (same four pointers) takes dt from those maxima alone
 * instead of re-reading the whole state.  dt is bitwise the one af_mhd_dt
 * computes from that state.  Contract: between the two calls the caller
 * does not change the state other than through af_mhd_step; a step on
 * another state or any af_mhd_stage call on the context falls back to the
 * full reduction.  Off by default. */
#define AF_FLAG_FUSED_DT 8u

typedef struct {            /* device time since init or the last reset */
  double ms_points;         /* point-value kernel (V, X, Y update) */
  double ms_cells;          /* cell-average kernel */
  double ms_dt;             /* time-step reduction */
  int64_t n_points, n_cells, n_dt;  /* launches timed */
} af_mhd_kernel_times_t;

typedef struct {            /* one state: the four DoF sets (layout above) */
  double* cell;
  double* xface;
  double* yface;
  double* vert;
} af_mhd_state;

typedef struct {
  double min_rho, min_p;    /* over all DoFs of the state */
  double mass;              /* sum of cell-average densities times dx dy */
  double min_theta;         /* smallest flux-limiter interface coefficient since init */
  int64_t n_llf_not_admissible; /* first-order LLF states outside G (Lemma's CFL violated) */
  int64_t n_newton;         /* vertex root solves of the flux limiter, step (2) */
  int64_t newton_iters_max;
  int64_t n_fallback;       /* round-off fallback uses (closing remark of Section 4) */
  int64_t n_not_admissible; /* stage outputs outside G */
  int64_t n_theta_active;   /* interfaces with a flux-limiter coefficient < 1 */
  int64_t n_point_limited;  /* point values changed by the scaling limiter */
  int64_t n_centre_limited; /* centre values changed by their limiter */
  int64_t n_source_limited; /* cells whose Powell source was blended towards LLF */
  int64_t n_dof_not_admissible; /* DoFs of the state passed to af_mhd_stats outside G */
} af_mhd_stats_t;

typedef struct af_mhd_ctx af_mhd_ctx;  /* opaque host object */

/* Bytes of device workspace the context needs for these parameters (RK
 * scratch states, stage intermediates, reduction buffers, counters).
 * Returns 0 for invalid parameters. */
size_t af_mhd_workspace_bytes(const af_mhd_params* p);

/* Create a context.  workspace_dev: caller-owned device buffer of at least
 * af_mhd_workspace_bytes(p) bytes, 256-byte aligned, kept alive until
 * af_mhd_destroy.  hip_stream: a hipStream_t (NULL = the null stream).
 * Zeroes the counters (asynchronously on the stream).  *out is set only on AF_OK. */
int af_mhd_init(const af_mhd_params* p, void* workspace_dev, size_t workspace_bytes, void* hip_stream,
                af_mhd_ctx** out);

/* Time step from the state u: dt = min(cfl / max_DoF(rho_1/dx + rho_2/dy),
 * t_remaining), written to dt_dev (one device double).  t_remaining > 0.
 * The paper states no time-step rule (a Lemma of Section 3.1 only bounds
 * the CFL number of its first-order scheme); this is the reading used:
 * rho_l = |v_l| + c_f,l, the spectral radius of dF_l/dU (Section 2.3), over
 * every cell average and point value. */
int af_mhd_dt(af_mhd_ctx* c, const af_mhd_state* u, double t_remaining, double* dt_dev);

/* One SSP-RK3 stage: out = a_k un + b_k FE(uk, dt) with (a,b) = (0,1),
 * (3/4,1/4), (1/3,2/3) for k = 0, 1, 2; FE is the limited forward-Euler step
 * of the scheme (Sections 2-3), dt read from dt_dev.  out must not alias uk;
 * out may alias un (each output element reads un only at its own index);
 * for k = 0 un is not read. */
int af_mhd_stage(af_mhd_ctx* c, int k, const af_mhd_state* un, const af_mhd_state* uk, af_mhd_state* out,
                 const double* dt_dev);

/* One SSP-RK3 step in place on u (SSP-RK3 of Section 2 in Shu-Osher form):
 * the time step, then the three stages af_mhd_stage k = 0, 1, 2, using the
 * workspace's scratch states.  The paper gives no time-step rule; the
 * reading used is dt = min(cfl / max over all DoFs of (rho_1/dx +
 * rho_2/dy), t_remaining) with rho_l = |v_l| + c_f,l (eq. (cf)), from U^n
 * and fixed over the three stages (as af_mhd_dt).  With AF_FLAG_FUSED_DT
 * the maximum comes from the previous step's last stage (see there).  The
 * dt used is left in dt_dev.  t_remaining > 0. */
int af_mhd_step(af_mhd_ctx* c, af_mhd_state* u, double t_remaining, double* dt_dev);

/* Statistics of u and the counters accumulated since af_mhd_init.
 * Synchronises the stream.  Returns AF_ENOTADMISSIBLE (with *out filled)
 * when some DoF of u is outside G. */
int af_mhd_stats(af_mhd_ctx* c, const af_mhd_state* u, af_mhd_stats_t* out);

/* The two discrete divergences the paper records for the Orszag-Tang
 * example (Section 4) of the state u, written to divb_dev[0..1] (device):
 *   div1 = sum over cells and the nine quadrature points of |div B| w_a w_b dx dy,
 *          div B as in the source of eq. (semi_av_src) (limited centre value);
 *   div2 = sum over cells of |Simpson edge integral of B.n| / 6 * dx dy, as printed.
 * Enqueued only; summed in a fixed order (bitwise reproducible). */
int af_mhd_divb(af_mhd_ctx* c, const af_mhd_state* u, double* divb_dev);

/* Reset the counters to zero (asynchronously on the stream). */
int af_mhd_reset_counters(af_mhd_ctx* c);

/* Per-kernel device time of a context created with AF_FLAG_KERNEL_TIMING
 * (AF_EINVAL otherwise).  Synchronises the stream.  reset != 0 zeroes the
 * totals after reading them.  Not a step of the method: a measurement aid. */
int af_mhd_kernel_times(af_mhd_ctx* c, af_mhd_kernel_times_t* out, int reset);

void af_mhd_destroy(af_mhd_ctx* c);

/* A plain device-to-device copy of n doubles (src, dst 16-byte aligned, n
 * even), enqueued on hip_stream: the project's own stream-copy kernel, the
 * attainable-bandwidth reference the stage kernels are compared with.  Not a
 * step of the method: a measurement aid.  AF_EINVAL on bad pointers or odd n. */
int af_mhd_stream_copy(const double* src, double* dst, size_t n, void* hip_stream);

/* ------------------------------------------------------------ limiters
 * The stage's positivity limiters applied to n given inputs, one device
 * thread per item, with the same device code the stage kernels run:
 *   AF_LIM_POINT   scaling limiter of a point value (Section 3.3):
 *                  in [n][16] = (U^H, U^LLF), out [n][8] = limited value
 *   AF_LIM_CENTRE  limiter of the centre value towards the cell average
 *                  (remark rmk:cell_center; one coefficient for the whole
 *                  state, density step then pressure step):
 *                  in [n][16] = (centre value, cell average), out [n][8]
 *   AF_LIM_SOURCE  step (1) of the parametrized flux limiter (Section 3.2):
 *                  in [n][25] = (G, S^s, S^LLF, dt) with A^LLF = G - dt S^LLF,
 *                  A^src = G - dt S^s; out [n][9] = (A^{Lim,1}, theta_src)
 *   AF_LIM_BOX     step (2): density box and the pressure shrink over the 15
 *                  non-trivial vertices; in [n][42] = (A^{Lim,1}, H_L, H_R,
 *                  H_D, H_U, eps_rho, eps_p), out [n][4] = Lambda_{L,R,D,U}
 * Each applies the round-off fallback of the closing remark of Section 4
 * (coefficient shrunk by 2^m 1e-8, m = 0..9, each trial from the original
 * value, floored at 0, when the limited state falls outside G).  Limiter
 * coefficients and every in-G decision use p = (gamma-1)(E - |m|^2/(2 rho)
 * - |B|^2/2) summed left to right without fused multiply-adds, so identical
 * inputs give a reference's results bit for bit.  AF_LIM_NO_SHORTCUT (box
 * only): test all 15 vertices even where the sufficient convexity test
 * (A^{Lim,1} and the four points A^{Lim,1} + 4 Lambda^rho_I H_I admissible)
 * already shows that none needs a root, as a reference without that test
 * does.  gamma > 1.  in_dev, out_dev: device arrays (doubles, 8-byte
 * aligned, caller-owned); counts_dev: device counters, added to (zero them
 * first).  Enqueued on hip_stream; AF_EINVAL for a bad kind, flag, size or
 * pointer, AF_EHIP if the launch fails.  A verification aid, not a step of
 * the method. */
enum { AF_LIM_POINT = 0, AF_LIM_CENTRE = 1, AF_LIM_SOURCE = 2, AF_LIM_BOX = 3 };
#define AF_LIM_NO_SHORTCUT 1u
typedef struct {            /* device counters (the stage's own, in this order) */
  int64_t n_llf_not_admissible, n_newton, newton_iters_max, n_fallback, n_not_admissible, n_theta_active,
      n_point_limited, n_centre_limited, n_source_limited, min_theta_bits;
} af_mhd_counters_t;
int af_mhd_limiters_apply(int kind, int64_t n, double gamma, const double* in_dev, double* out_dev, uint32_t flags,
                          af_mhd_counters_t* counts_dev, void* hip_stream);

/* One SSP-RK3 step in place on u, as af_mhd_step on a context created
 * with these parameters, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): no context, no workspace and no allocation of any kind.  Its
 * scratch (the workspace of af_mhd_step) lives in a 48 MiB file-scope
 * device array that every GPU the library runs on holds until the process
 * ends; grids whose workspace exceeds it (beyond about 256 x 256 cells) are
 * rejected with AF_EINVAL.  Every call on one GPU shares that GPU's array:
 * calls that overlap on one GPU (other streams, other threads) race and
 * must not be issued.  The limiter counters restart from zero on every call
 * and are not reported.  p->flags: AF_FLAG_FP32_BULK only.  Enqueued on
 * hip_stream; dt is left in dt_dev.  Errors: AF_EINVAL for bad parameters,
 * pointers or sizes, AF_EHIP for a HIP failure; the message is that of
 * af_mhd_last_error(NULL) on this thread. */
int af_mhd_step_noalloc(const af_mhd_params* p, af_mhd_state* u, double t_remaining, double* dt_dev,
                        void* hip_stream);

/* ------------------------------------------------------------ batches
 * A batch advances n independent grids together (each with its own
 * parameters: sizes, domain, gamma, cfl, kappa, boundaries; the flags must
 * agree).  Per SSP-RK3 step it runs one launch computing every instance's
 * dt (min(cfl / max wave speed, t_remaining)), then per stage, by launch
 * mode (af_mhd_batch_set_launch_mode):
 *   AF_BATCH_FUSED       one launch over the point tiles of all instances
 *                        (two per 512-thread workgroup) and their cell tiles,
 *                        which compute their cells' nine-point sources
 *                        themselves, so that no workgroup waits on another;
 *   AF_BATCH_PERSISTENT  one launch of the point update over the (instance,
 *                        tile) work items of all instances and one of the
 *                        cell update over theirs, persistent workgroups;
 *   AF_BATCH_FLAT        the same two launches, one item per workgroup.
 * Cell tiles are 32 x 16 or 16 x 32: the shape tuned for the size classes
 * holding most of the batch's cells.  The step can be captured once into a
 * hipGraph and replayed.  Each instance's results are bitwise equal to
 * what a single-grid context computes on it, in every mode. */
typedef struct af_mhd_batch af_mhd_batch;

#define AF_BATCH_FLAT 0
#define AF_BATCH_PERSISTENT 1
#define AF_BATCH_FUSED 2

/* Bytes of device workspace for n instances with parameters p[0..n-1]
 * (two RK scratch states and a nine-point source buffer per instance, dt partials,
 * counters, launch tables).  0 for invalid parameters or mixed flags. */
size_t af_mhd_batch_workspace_bytes(const af_mhd_params* p, int n);

/* Create a batch bound to the caller's states[0..n-1] (layout as above;
 * stepped in place), dt_dev (n device doubles, written every step),
 * t_remaining_dev (n device doubles read every step, or NULL for no end
 * time) and workspace (256-byte aligned, af_mhd_batch_workspace_bytes).
 * All must stay valid until af_mhd_batch_destroy.  tune_table: path of a
 * text table of cell-tile shapes per size class ("nx ny bc_x bc_y
 * fp64|fp32 shape" lines); classes missing from it are measured on the
 * device (a few launches on the first instance of the class, which
 * compute into the scratch states only) and appended.  NULL: the default
 * 32x16 tile for every instance.  Synchronises the stream. */
int af_mhd_batch_init(const af_mhd_params* p, int n, const af_mhd_state* states, double* dt_dev,
                      const double* t_remaining_dev, void* workspace_dev, size_t workspace_bytes, void* hip_stream,
                      const char* tune_table, af_mhd_batch** out);

/* One SSP-RK3 step of every instance, enqueued on the batch's stream.
 * use_graph != 0: the first call captures the step into a hipGraph, every
 * call launches the graph; 0: plain launches. */
int af_mhd_batch_step(af_mhd_batch* b, int use_graph);

/* Cell-tile shape (threads in x and y) of the batch's cell launch, which
 * instance m runs on (the same for every m). */
int af_mhd_batch_tile(const af_mhd_batch* b, int m, int* tile_x, int* tile_y);

/* Launch mode of the stages (AF_BATCH_FLAT, AF_BATCH_PERSISTENT or
 * AF_BATCH_FUSED, described above) into *mode.  AF_BATCH_FLAT by default;
 * with a tune table, the fastest of the three on this batch (measured at
 * init on stage-0 launches). */
int af_mhd_batch_launch_mode(const af_mhd_batch* b, int* mode);

/* Set the launch mode of the following steps (a graph captured in another
 * mode is dropped and the next graph step captures anew).  AF_EINVAL for
 * an unknown mode. */
int af_mhd_batch_set_launch_mode(af_mhd_batch* b, int mode);


/* Limiter counters accumulated over all instances since init (the state
 * statistics fields of out are left zero).  Synchronises the stream. */
int af_mhd_batch_counters(af_mhd_batch* b, af_mhd_stats_t* out);

void af_mhd_batch_destroy(af_mhd_batch* b);

/* Message of the last error on this batch; with b == NULL, of this
 * thread's last failed af_mhd_batch_init. */
const char* af_mhd_batch_last_error(const af_mhd_batch* b);

/* Message of the last error on this context ("" if none); valid until the
 * next call.  With c == NULL: the message of this thread's last failed
 * af_mhd_init. */
const char* af_mhd_last_error(const af_mhd_ctx* c);

/* ------------------------------------------------------------ adjoint
 * Discrete adjoint of one SSP-RK3 stage out = a_k un + b_k FE(uk, dt): the
 * transposed Jacobian of the stage of Sections 2-3 with dt fixed and every
 * decision of the positivity limiters (Sections 3.2, 3.3, the remark on the
 * centre value and the round-off fallback of Section 4) and of the shock
 * sensor (Section 3.4) frozen as the recorded forward took it.  Within a
 * decision the derivative is exact: guarded fractions, the density box, the
 * vertex roots (implicit derivative of the pressure condition along the
 * ray), the sensor's exp/max terms and the LLF viscosities (largest of the
 * Lemma's four speeds) are differentiated.  Conventions: max/min ties go to
 * the first argument, |x| has derivative +1 at 0, sqrt derivative 0 at 0.
 * FP64 only (params->flags must be 0).  The state layout is the one above.
 * Work is enqueued on the context's stream; nothing synchronises. */
typedef struct af_mhd_adj af_mhd_adj;  /* opaque host object */

/* Bytes of one stage's tape (decisions, limiter coefficients and roots,
 * interface fluxes, sources, centre values), about 110 doubles per cell.
 * 0 for invalid parameters. */
size_t af_mhd_adj_tape_bytes(const af_mhd_params* p);

/* Bytes of the adjoint context's device workspace (adjoints of the stage's
 * intermediate quantities).  0 for invalid parameters. */
size_t af_mhd_adj_workspace_bytes(const af_mhd_params* p);

/* Create an adjoint context; workspace_dev: caller-owned, 256-byte
 * aligned, at least af_mhd_adj_workspace_bytes(p), kept until destroy. */
int af_mhd_adj_init(const af_mhd_params* p, void* workspace_dev, size_t workspace_bytes, void* hip_stream,
                    af_mhd_adj** out);

/* Recording forward stage: writes out = a_k un + b_k FE(uk, dt) (the same
 * stage as af_mhd_stage, evaluated entity by entity in the paper's order
 * with IEEE division; equal to it to rounding) and the stage's tape into
 * tape_dev (caller-owned device buffer, 256-byte aligned, at least
 * af_mhd_adj_tape_bytes).  out must not alias uk; un is not read for k = 0. */
int af_mhd_adj_record(af_mhd_adj* c, int k, const af_mhd_state* un, const af_mhd_state* uk, af_mhd_state* out,
                      const double* dt_dev, void* tape_dev, size_t tape_bytes);

/* Reverse sweep of the recorded stage k with input uk and tape_dev:
 *   lam_n += a_k lam_out   and   lam_k += b_k (dFE/duk)^T lam_out,
 * lam_out being the adjoint of the stage output.  The accumulators are
 * added to (zero them first for a fresh gradient).  For k = 0 (a_0 = 0)
 * lam_n is not touched and may be NULL or equal to lam_k.  lam_out must not
 * alias an accumulator.  Sums use device atomics: the result is not
 * bitwise reproducible run to run (rounding-level differences only). */
int af_mhd_adj_stage(af_mhd_adj* c, int k, const af_mhd_state* uk, const void* tape_dev, size_t tape_bytes,
                     const double* dt_dev, const af_mhd_state* lam_out, af_mhd_state* lam_n, af_mhd_state* lam_k);

void af_mhd_adj_destroy(af_mhd_adj* c);

/* Message of the last error on this adjoint context; with c == NULL, of
 * this thread's last failed af_mhd_adj_init. */
const char* af_mhd_adj_last_error(const af_mhd_adj* c);

#ifdef __cplusplus
}
#endif
#endif /* AF_MHD_H */
