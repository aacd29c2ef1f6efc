/*
 * mstar.h -- C ABI of the MI355X (gfx950) FP64 implementation of the MSTAR
 * algorithmically regularised integrator with minimum-spanning-tree
 * coordinates (Rantala, Pihajoki, Mannerkoski, Johansson & Naab 2020).
 *
 * The problem statement follows the paper (Sec. 2.4): masses, positions and
 * velocities at t0 in, the state at t_end out, with the GBS tolerance eta
 * (eq. gbs-criterion) as the accuracy parameter.  Every step of the method
 * runs in this library's HIP kernels; the host only sequences launches and
 * makes the accept/halve decision from a few scalars read back per step.
 *
 * Conventions for every entry point:
 *  - FP64 throughout; G = params->G.
 *  - Array arguments are caller-owned, read or written only during the call,
 *    never retained.  With MSTAR_DEVICE_PTRS in params->flags (or the
 *    `flags` argument of a stage call) they are device pointers on the
 *    context's device (e.g. contiguous float64 torch tensors); otherwise host
 *    pointers.  Vectors are [n][3] row-major (x, y, z of body i at 3i..3i+2).
 *  - MST state arrays: parent[n] (int32, the root has -1); X[n][3], V[n][3]
 *    with row v holding the edge vector from parent(v) to v (root row 0).
 *  - Return value: MSTAR_OK (0), a negative MSTAR_E_* code, or the positive
 *    warning MSTAR_W_TIME_TOL.  Validation errors leave outputs untouched;
 *    runtime errors of mstar_integrate leave the last accepted state in x, v
 *    with stats->t_reached set.  No exception or abort crosses the ABI.
 *  - A context is not thread-safe; distinct contexts are independent.  Work
 *    is enqueued on the context's stream; calls return after completion.
 *  - Same inputs, parameters and device give bitwise identical outputs.
 */
#ifndef MSTAR_H
#define MSTAR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MSTAR_ABI_VERSION 2

#define MSTAR_OK 0
#define MSTAR_E_INVAL -1       /* invalid argument or parameter */
#define MSTAR_E_NOMEM -2       /* device or host allocation failed */
#define MSTAR_E_DEVICE -3      /* HIP runtime error */
#define MSTAR_E_NONFINITE -4   /* NaN/Inf in the inputs */
#define MSTAR_E_COINCIDENT -5  /* two bodies at the same position */
#define MSTAR_E_NOCONV -6      /* GBS did not converge within max_halvings */
#define MSTAR_E_MAXSTEPS -7    /* max_steps GBS steps taken before t_end */
#define MSTAR_E_UNSUPPORTED -8 /* valid for the method but not implemented here */
#define MSTAR_W_TIME_TOL 1     /* t_end not met within t_tol after max_time_iter clipped steps */

#define MSTAR_DEVICE_PTRS 1u   /* array arguments are device pointers */
#define MSTAR_EAGER 2u         /* mstar_integrate*: launch each GBS step attempt's kernels from
                                  the host instead of replaying the attempt as a captured HIP
                                  graph (same kernels, same order, identical results) */
#define MSTAR_MST_DC 4u        /* mstar_mst_build and the single-system integrators: build every
                                  spanning tree by the divide-and-conquer method of Sec. 3.3
                                  (octree groups of at most ceil(sqrt(N)) bodies, the minimum
                                  spanning tree of each group and of the meta-graph of groups)
                                  instead of the exact MST.  Ignored by the batched integrator. */

/* Parameters of the method.  struct_size must be sizeof(mstar_params);
 * mstar_params_default fills every field. */
typedef struct {
    uint32_t struct_size;
    uint32_t flags;         /* MSTAR_DEVICE_PTRS | MSTAR_EAGER */
    double G;               /* gravitational constant (Sec. 2.1) */
    double eta;             /* GBS tolerance eta_GBS, eq. gbs-criterion; default 1e-12 */
    double alpha, beta, gamma; /* time-transformation triplet, eq. ttl; default LogH (1,0,0) */
    double omega_mass_max;  /* TTL Omega couples bodies with m <= this (beta != 0) */
    double a_gbs;           /* safety factor of eq. hnext, in (0, 1]; default 0.9.  Runs settle at
                               eps ~ eta a_gbs^(2 k_fix - 1); measured to take the least work:
                               1.0 at eta <= 1e-12, 0.85 near 1e-10, 0.6 near 1e-6 (7-12% fewer
                               force evaluations than 0.9).  Below 0.8 at eta <= 1e-12 the target
                               falls under the rounding floor of eps and the steps collapse. */
    double f_min, f_max;    /* clamps of the eq. hnext step ratio; default 0.1, 4 */
    double q_first;         /* first step ds = q U dt (Sec. 2.4); default 0.1 */
    double t_tol;           /* stop when |t_end - t| <= t_tol |t_end - t0|; default 1e-14 */
    double h_init;          /* > 0: first fictitious step; 0: automatic */
    int64_t max_steps;      /* GBS step attempts (accepted + rejected) */
    int32_t k_fix;          /* substep divisions n_k = 2k, k = 1..k_fix (Sec. 4.2); 2..16, default 8 */
    int32_t n_d;            /* MST closeness N_d of eq. LCA; 0..4 here (0..2 in the batch kernel), default 2 */
    int32_t max_halvings;   /* consecutive rejections before MSTAR_E_NOCONV; default 60 */
    int32_t max_time_iter;  /* clipped end-time steps before MSTAR_W_TIME_TOL; default 8 */
    int32_t rebuild_every;  /* accepted steps between MST rebuilds (Sec. 3.5); default 1 */
    int32_t accept_rule;    /* where eq. gbs-criterion is judged: 0 (default) at k_fix, the fixed
                               division count of Sec. 4.2, returning T_{k_fix,k_fix}; 1 at the first
                               k = 2..k_fix whose error measure eps_k <= eta (the serial rule of
                               Sec. 2.3), returning T_{k,k} and taking eq. hnext with that k.  All
                               k_fix divisions are computed either way.  Not in the batch kernel. */
} mstar_params;

/* Per-call statistics. */
typedef struct {
    uint32_t struct_size;
    uint32_t reserved;
    int64_t steps_accepted, steps_rejected;
    int64_t force_evals;    /* full O(N^2) force evaluations */
    int64_t mst_rebuilds, topo_changes, time_iters;
    double t_reached;       /* physical time of the returned state */
    double eps_last;        /* error measure of the last GBS step */
    double h_next;          /* suggested next fictitious step (pass as h_init to continue) */
    double h_last;          /* last accepted fictitious step */
} mstar_stats;

typedef struct mstar_ctx mstar_ctx;

/* Version of this ABI (MSTAR_ABI_VERSION). */
int mstar_abi_version(void);

/* Fill *p with the defaults listed above; sets p->struct_size. */
void mstar_params_default(mstar_params *p);

/* Static string for a return code. */
const char *mstar_strerror(int code);

/* Create a context on HIP device `hip_device`.  `hip_stream` is a hipStream_t
 * to enqueue work on, or NULL for a stream owned by the context.  Device
 * scratch is allocated on demand and kept until mstar_destroy.  The
 * integration calls capture their GBS step attempts on this stream as HIP
 * graphs and replay them (unless MSTAR_EAGER); a stream that cannot be
 * captured makes the context launch directly instead.
 * Errors: MSTAR_E_INVAL (bad device), MSTAR_E_DEVICE, MSTAR_E_NOMEM. */
int mstar_create(mstar_ctx **out, int hip_device, void *hip_stream);

/* Free the context and its device memory.  NULL is allowed. */
void mstar_destroy(mstar_ctx *ctx);

/* Message of the last error on ctx (context-owned, valid until the next call). */
const char *mstar_last_error(const mstar_ctx *ctx);

/* Integrate n bodies from t0 to t_end (paper Sec. 2.4 driver; Sec. 2.3 GBS
 * with the Deuflhard sequence; Sec. 3 MST coordinates).  x, v [n][3] are read
 * at t0 and overwritten with the state at stats->t_reached.  m [n] > 0.
 * Errors: MSTAR_E_INVAL (n < 2, bad masses or parameters), MSTAR_E_NONFINITE,
 * MSTAR_E_COINCIDENT, MSTAR_E_NOCONV, MSTAR_E_MAXSTEPS, MSTAR_E_UNSUPPORTED
 * (n_d > 4), device errors; warning MSTAR_W_TIME_TOL.  With beta != 0 the
 * time transformation includes the TTL function Omega of Sec. 2.1 over the
 * bodies with m <= omega_mass_max, and its auxiliary variable w starts at
 * Omega(t0); alpha = gamma = 0 then needs at least two such bodies
 * (MSTAR_E_INVAL otherwise). */
int mstar_integrate(mstar_ctx *ctx, const mstar_params *params, int64_t n, const double *m,
                    double *x, double *v, double t0, double t_end, mstar_stats *stats);

/* External perturbation of the N-body system (Sec. 2.1: a position-dependent
 * acceleration f_i(r_i) added to the Newtonian one).  The field offered:
 *   f(r) = g + G sum_k M_k (R_k - r) / (|R_k - r|^2 + b_k^2)^(3/2),
 * a uniform acceleration plus n_point fixed Plummer-softened point masses,
 * point[k] = {M_k, X_k, Y_k, Z_k, b_k} in host memory (M_k >= 0, b_k >= 0;
 * b_k = 0 is a bare point mass).  Caller-owned; read during the call only. */
#define MSTAR_MAX_EXT_POINTS 16
typedef struct {
    uint32_t struct_size;      /* sizeof(mstar_external) */
    int32_t n_point;           /* 0 .. MSTAR_MAX_EXT_POINTS */
    double g[3];
    const double *point;       /* [n_point][5], may be NULL when n_point = 0 */
} mstar_external;

/* mstar_integrate under the external field *ext (Sec. 2.1).  Each kick adds
 * f_i to every body's acceleration and to the centre-of-mass velocity (as
 * F/M, F = sum m_i f_i); since f is constant over a kick, the binding energy
 * B = -(T - U) of the internal motion takes the field's work exactly,
 * B -= dt sum_i m_i f_i . (v_i_old + v_i_new)/2 with centre-of-mass-frame
 * velocities.  B and v_cm are extrapolated and error-tested with the rest of
 * the state.  Arguments, layout, ownership and errors as mstar_integrate, and
 * MSTAR_E_INVAL for a NULL, wrongly sized or non-finite field, a negative
 * mass or softening, or n_point out of range; MSTAR_E_UNSUPPORTED with
 * beta != 0.  A body exactly on an unsoftened point mass makes f infinite;
 * the step then fails to converge (MSTAR_E_NOCONV). */
int mstar_integrate_ext(mstar_ctx *ctx, const mstar_params *params, int64_t n, const double *m,
                        double *x, double *v, double t0, double t_end, const mstar_external *ext,
                        mstar_stats *stats);

/* ---- stage entry points (each is one row of the method; used by parity
 * tests, the benchmark and callers that drive the steps themselves) ---- */

/* Minimum spanning tree (Sec. 3.1-3.4) of the complete graph on positions
 * x [n][3] under the strict edge order (w = |x_j - x_i|^2 evaluated as
 * (dx*dx + dy*dy) + dz*dz without fused multiply-add, then min index, then max
 * index), rooted at the body nearest the centre of mass of masses m (ties to
 * the lowest index), or at `root_in` if 0 <= root_in < n.  Outputs parent[n]
 * (root -1), level[n] (root 0) and *root_out.  Host or device pointers per
 * `flags`.  With MSTAR_MST_DC in `flags` the tree is the divide-and-conquer
 * spanning tree of Sec. 3.3 instead (same root rule): the bounding cube of x
 * (lower corner the per-axis minimum, side the largest extent) is split as an
 * octree, each cell holding more than ceil(sqrt(n)) bodies into its octants
 * down to 10 levels, every non-empty unsplit cell is a group, and the tree is
 * the union of each group's MST and of the MST of the meta-graph whose edge
 * between two groups is their lightest connecting edge (all under the strict
 * order above). */
int mstar_mst_build(mstar_ctx *ctx, uint32_t flags, int64_t n, const double *m, const double *x,
                    int32_t root_in, int32_t *parent, int32_t *level, int32_t *root_out);

/* Accelerations and force function with MST separations (Sec. 2.1 and the
 * close-pair rule of Sec. 3.4): acc[n][3] = G sum_j m_j d_ij/|d_ij|^3 and
 * *U = G sum_{i<j} m_i m_j/|d_ij|, where d_ij is the MST path sum of the edge
 * vectors X for pairs within params->n_d tree edges and rho_j - rho_i
 * otherwise.  rho [n][3] are positions in any frame consistent with X.
 * Omega and dOmega may be NULL.  With params->beta != 0 they receive the TTL
 * function Omega = G sum_{i<j} mo_i mo_j/|d_ij| and its gradient
 * dOmega[i] = G mo_i sum_j mo_j d_ij/|d_ij|^3, where mo_i = m_i if
 * m_i <= omega_mass_max, else 0.  With beta == 0 they receive zeros. */
int mstar_force(mstar_ctx *ctx, const mstar_params *params, int64_t n, const double *m,
                const double *rho, const int32_t *parent, const double *X, double *acc, double *U,
                double *Omega, double *dOmega);

/* One leapfrog division over the fictitious interval H with nsub substeps,
 * D(H/2n)[K(H/n)D(H/n)]^(n-1)K(H/n)D(H/2n) (Sec. 2.3), on the MST state
 * (parent, X, V) with scal[9] = (t, B, w, r_cm[3], v_cm[3]); X, V, scal are
 * updated in place.  B must be the binding energy -H of the state. */
int mstar_leapfrog(mstar_ctx *ctx, const mstar_params *params, int64_t n, const double *m,
                   const int32_t *parent, double *X, double *V, double *scal, double H, int32_t nsub);

/* One GBS step of fictitious length H (Sec. 2.3, 4.2): k_fix divisions from
 * the same start state, Neville-Aitken extrapolation, error test.  If
 * *accepted, X, V, scal hold the extrapolated state; otherwise they are
 * unchanged.  *eps is the error measure, *h_next the next step (eq. hnext on
 * acceptance, H/2 on rejection).  No MST rebuild is done here. */
int mstar_gbs_step(mstar_ctx *ctx, const mstar_params *params, int64_t n, const double *m,
                   const int32_t *parent, double *X, double *V, double *scal, double H,
                   int32_t *accepted, double *eps, double *h_next);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid it): mstar_force without a
 * context and without any allocation, host copy or synchronisation.  The
 * work is only enqueued on hip_stream (a hipStream_t; NULL: the null stream)
 * of the current device; outputs are valid once that stream has reached this
 * point.  m [n], rho [n][3], parent [n] (int32), X [n][3] are device
 * pointers read by the enqueued kernels, acc [n][3] and U (one double) device
 * pointers written by them; parent, X, rho and the result as mstar_force
 * (params->n_d 0..4, params->beta must be 0; params->flags is ignored).  The
 * library keeps its intermediate results in a fixed device array of about
 * 6 MB per device (allocated with the library's code object, not by the
 * call), so n is limited to MSTAR_NOALLOC_MAX_N, and calls that overlap on one
 * device (different streams or host threads) race on that array.  Errors:
 * MSTAR_E_INVAL (NULL pointers, bad params, n < 2 or n > MSTAR_NOALLOC_MAX_N),
 * MSTAR_E_UNSUPPORTED (n_d > 4, beta != 0), MSTAR_E_DEVICE.  A parent array
 * that is not one rooted tree cannot be reported synchronously: acc and U
 * are then NaN. */
#define MSTAR_NOALLOC_MAX_N 8192
int mstar_force_noalloc(void *hip_stream, const mstar_params *params, int64_t n, const double *m, const double *rho,
                        const int32_t *parent, const double *X, double *acc, double *U);

/* Force-kernel timing for measurement: when enabled, every force-kernel
 * launch is bracketed by HIP events on the stream it runs on; the totals cover
 * all launches since the last reset.  kernel_ms is the time during which any
 * of them ran: the union of their intervals (the launches of two concurrent
 * division chains overlap; for launches on one stream it is the sum of their
 * durations), placed by float-millisecond offsets from the enable call
 * (resolution about 1e-7 of the profiling window).  A batched call counts as
 * one launch (the persistent batch kernel) with the pair interactions of all
 * its force evaluations. */
int mstar_profile_enable(mstar_ctx *ctx, int enable);
int mstar_profile_read(mstar_ctx *ctx, int64_t *launches, double *kernel_ms, double *pairs);
/* The same totals for one force kernel: kind 0 the pairwise kernel (each
 * directed pair formed by its receiving body), 1 the mutual kernel (each
 * unordered pair once, applied to both bodies).  Batched launches are not
 * included.  Errors: MSTAR_E_INVAL for another kind. */
int mstar_profile_read_kernel(mstar_ctx *ctx, int32_t kind, int64_t *launches, double *kernel_ms, double *pairs);

/* Coordinate round trips (Sec. 3.5): for each of n_sys systems (bodies
 * offsets[s] .. offsets[s+1]-1, 2 <= N <= 512), n_cycles times: build the
 * coordinate structure from the Cartesian state -- kinds[s] = 0: the MST of
 * Sec. 3.1-3.4 rooted at the body nearest the centre of mass; 1: the chain of
 * Sec. 2.2 (the ends of the shortest edge start it, the body nearest either
 * end joins there; edges compared under the strict order of the MST, the
 * lower-indexed end of the first edge is the first tail) -- form the edge
 * vectors and the centre of mass, and rebuild x, v from them (x = r_cm +
 * (rho - rho_bar), rho the root-relative path sums).  Centre-of-mass sums
 * are compensated (Neumaier); kinds 2 and 3 are kinds 0 and 1 with plain
 * sums in index order instead (the paper's test, Sec. 3.5, does not
 * compensate).  The inputs x, v
 * ([n_tot][3]) are not modified; after cycle (k+1) n_cycles / n_out the state
 * is written to x_out[k], v_out[k] ([n_out][n_tot][3]).  mean_level (host,
 * nullable, [n_sys]) receives the structure's mean body level averaged over
 * the cycles (a chain's is (N-1)/2).  Pointers per `flags` except mean_level.
 * Errors: MSTAR_E_INVAL, MSTAR_E_NOMEM, device errors. */
int mstar_rebuild_cycles(mstar_ctx *ctx, uint32_t flags, int32_t n_sys, const int64_t *offsets,
                         const int32_t *kinds, const double *m, const double *x, const double *v,
                         int64_t n_cycles, int32_t n_out, double *x_out, double *v_out, double *mean_level);

/* Measurement aid for the force loop's roofline: SIMD cycles per wave-level
 * FP64 fused multiply-add (*fma_cycles) and per hardware 1/sqrt
 * (*rsq_cycles), from chip-wide streams of independent instructions timed
 * with HIP events and expressed at the nominal 2.4 GHz clock (4 cycles per
 * FMA at that clock is the nominal FP64 peak).  Allocates and frees 4 MiB of
 * device memory; takes a few milliseconds.  Errors: MSTAR_E_INVAL, device
 * errors. */
int mstar_issue_rates(mstar_ctx *ctx, double *fma_cycles, double *rsq_cycles);

/* ---- many independent small systems in one launch ----
 * The method applied to n_sys independent systems at once (Sec. 4.2 notes the
 * extension to several independent systems); each system is integrated
 * exactly as by mstar_integrate (same driver, GBS step, MST rebuilds and
 * arithmetic), all of them inside one persistent kernel launched through a
 * captured HIP graph. */

/* Per-system outcome of a batched call. */
typedef struct {
    int32_t status;         /* MSTAR_OK, MSTAR_W_TIME_TOL or a negative code, as mstar_integrate returns */
    int32_t reserved;
    int64_t steps_accepted, steps_rejected;
    int64_t force_evals, mst_rebuilds, topo_changes, time_iters;
    double t_reached, eps_last, h_next, h_last;
} mstar_batch_stats;

/* Launch shape of the batch kernel (one per k_fix, kept in the context).
 * Systems with N > wave_max_n are integrated by a whole 256-thread workgroup
 * (bodies on 64 lanes, one division pair (n, 2 k_fix + 2 - n) per wave);
 * systems with N <= wave_max_n by a single wave whose lanes form 64/wave_lanes
 * groups of wave_lanes lanes, each group running division pairs. */
typedef struct {
    uint32_t struct_size;
    int32_t wave_lanes;     /* 0 (no single-wave systems), 16, 32 or 64 */
    int32_t wave_max_n;     /* 0..wave_lanes */
    int32_t wgs_per_cu;     /* persistent workgroups per compute unit; 0 = as many as fit */
    int32_t use_graph;      /* 1: launch through a captured HIP graph (default); 0: plain launch */
    int32_t reserved;
    double kernel_ms;       /* mstar_batch_autotune: time of the chosen shape; else 0 */
} mstar_batch_config;

/* Integrate system s (bodies offsets[s] .. offsets[s+1]-1) from t0[s] (0 if t0
 * is NULL) to t_end[s], for s < n_sys.  m [N], x, v [N][3] with N =
 * offsets[n_sys] follow params->flags (host or device) and x, v are
 * overwritten with each system's end state (where its status is OK,
 * W_TIME_TOL, NOCONV or MAXSTEPS).  offsets [n_sys+1] (int64, offsets[0] = 0),
 * t0, t_end [n_sys] and stats [n_sys] are host memory.  Every system has
 * N_s >= 2 bodies.  Systems with N_s <= 64 run in the persistent launch;
 * larger ones are integrated after it, one after the other, by
 * mstar_integrate's driver (the same results as a mstar_integrate call, their
 * own status in stats).  Parameters the persistent kernel does not implement
 * (k_fix > 8, beta != 0, n_d > 2, accept_rule 1) send every system through
 * that driver, so the call takes the parameter sets mstar_integrate takes.
 * Returns MSTAR_OK when the call completed (per-system results in stats),
 * MSTAR_E_INVAL (bad offsets, times or parameters), MSTAR_E_UNSUPPORTED
 * (as mstar_integrate: n_d > 4) or a device error. */
int mstar_integrate_batch(mstar_ctx *ctx, const mstar_params *params, int32_t n_sys, const int64_t *offsets,
                          const double *m, double *x, double *v, const double *t0, const double *t_end,
                          mstar_batch_stats *stats);

/* mstar_integrate_batch that also records the fictitious step H of every
 * accepted step of every system: H [n_sys][rec_cap] (host memory; row s
 * holds system s's first min(stats[s].steps_accepted, rec_cap) steps, the
 * rest of the row is NaN).  The record lets a system be replayed step for step (as
 * mstar_integrate_record does for one system).  Errors as
 * mstar_integrate_batch, and MSTAR_E_INVAL for a NULL H or rec_cap < 1. */
int mstar_integrate_batch_record(mstar_ctx *ctx, const mstar_params *params, int32_t n_sys, const int64_t *offsets,
                                 const double *m, double *x, double *v, const double *t0, const double *t_end,
                                 mstar_batch_stats *stats, int64_t rec_cap, double *H);

/* Read or replace the launch shape used for k_fix (2..8). */
int mstar_batch_get_config(mstar_ctx *ctx, int32_t k_fix, mstar_batch_config *cfg);
int mstar_batch_set_config(mstar_ctx *ctx, int32_t k_fix, const mstar_batch_config *cfg);

/* Autotuner: time every launch shape (wave_lanes, wave_max_n, wgs_per_cu)
 * on this batch (same arguments as mstar_integrate_batch; x and v are not
 * modified; pass a shortened t_end to bound the cost), keep the fastest for
 * params->k_fix in the context and return it in *best.  MSTAR_E_INVAL when
 * no system has at most 64 bodies (nothing runs in the kernel); MSTAR_E_UNSUPPORTED
 * for parameters the persistent kernel does not implement (k_fix > 8,
 * beta != 0, n_d > 2, accept_rule 1). */
int mstar_batch_autotune(mstar_ctx *ctx, const mstar_params *params, int32_t n_sys, const int64_t *offsets,
                         const double *m, const double *x, const double *v, const double *t0,
                         const double *t_end, mstar_batch_config *best);

/* ---- frozen-controller replay and adjoint (gradients of the end state with
 * respect to the initial conditions; not in the paper) ----
 * With the accepted fictitious steps H_k recorded, the integrator is a smooth
 * map from (x0, v0) to the end state (discretise, then differentiate: the
 * step-size controller is frozen).  In exact arithmetic that map does not
 * depend on the coordinates it is evaluated in (the MST transforms and
 * rebuilds of Sec. 2.2 and 3.5 are linear changes of variables), so the
 * replay and its adjoint evaluate it in Cartesian coordinates: the LogH
 * leapfrog of Sec. 2.1-2.3 with B = U(x0) - T(v0), and each GBS step the
 * k_fix divisions combined with the weights of the extrapolation to h = 0 in
 * h^2 (Sec. 2.3, 4.2).  N <= 1024 (MSTAR_E_UNSUPPORTED above), k_fix <= 16. */

/* mstar_integrate that records the fictitious step H[k] of every accepted
 * step (H has room for max_accepted values, host memory) and stops after
 * max_accepted accepted steps if t_end is not reached first (MSTAR_OK in
 * both cases); *n_accepted = steps recorded. */
int mstar_integrate_record(mstar_ctx *ctx, const mstar_params *params, int64_t n, const double *m, double *x,
                           double *v, double t0, double t_end, int64_t max_accepted, double *H,
                           int64_t *n_accepted, mstar_stats *stats);

/* Replay n_steps GBS steps of lengths H[k] (host array) from (x, v) at t0
 * without error test or step control; x, v are overwritten with the end
 * state and *t_out (nullable) receives its time. */
int mstar_replay(mstar_ctx *ctx, const mstar_params *params, int64_t n, const double *m, double *x, double *v,
                 double t0, int64_t n_steps, const double *H, double *t_out);

/* Adjoint of mstar_replay: given the cotangent (gx, gv [n][3], gt) of the end
 * state (x, v, t), returns gx0, gv0 = the gradient of <gx, x> + <gv, v> + gt t
 * with respect to the initial x0, v0, and (gm [n], nullable) with respect to
 * the masses m, which enter the accelerations, the force function U of the
 * kicks' time transformation, the kinetic energy T of the drifts' and the
 * binding energy B = U(x0) - T(v0).  Checkpoints the state every
 * checkpoint_every steps; the reverse pass recomputes one segment at a time
 * from its checkpoint, keeping the substep states of all its steps (blocks
 * of fewer steps if two segments' states exceed the context's store limit,
 * see mstar_adjoint_store_limit), on a second stream of the context's device
 * while the previous block is reversed on ctx's stream.  The result is
 * bitwise independent of checkpoint_every and of the store limit. */
int mstar_replay_adjoint(mstar_ctx *ctx, const mstar_params *params, int64_t n, const double *m, const double *x0,
                         const double *v0, double t0, int64_t n_steps, const double *H, int32_t checkpoint_every,
                         const double *gx, const double *gv, double gt, double *gx0, double *gv0, double *gm);

/* Upper bound, in bytes, of the device memory in which the reverse pass of
 * mstar_replay_adjoint / mstar_integrate_adjoint keeps recomputed substep
 * states (two blocks of steps; each step holds every kick's positions, every
 * drift's velocities and the op scalars of its k_fix divisions, about
 * 32 (2 k_fix^2 + 3 k_fix) N bytes).  0 restores the default of 4 GiB.  At
 * least two steps' states are always kept, whatever the limit.  The memory is
 * allocated on the next adjoint call that needs more than the context holds
 * and kept until mstar_destroy.  MSTAR_E_INVAL for bytes < 0. */
int mstar_adjoint_store_limit(mstar_ctx *ctx, int64_t bytes);

/* Record and reverse in one call: integrate from (x0, v0) at t0 toward t_end
 * (mstar_integrate's driver, Sec. 2.4) until n_steps steps are accepted or
 * t_end is reached, then return the gradient of <gxT, x> + <gvT, v> + gtT t
 * at the end state with respect to x0, v0 (gx0, gv0 [n][3]) and the masses
 * (gm [n], nullable), with the step sizes and MST topologies of the recorded
 * run frozen (as mstar_replay_adjoint).  The adjoint's checkpoint pass
 * replays each step on a second stream of the device as soon as the driver
 * has accepted it, alongside the integration; the result equals
 * mstar_integrate_record followed by mstar_replay_adjoint bit for bit.
 * x0, v0 are not modified; stats
 * (nullable) receives the forward run's statistics (its steps_accepted is
 * the number of steps differentiated).  Pointers per params->flags.
 * Errors: MSTAR_E_INVAL, MSTAR_E_UNSUPPORTED (n > 1024, beta != 0), the
 * integrator's errors (the gradient is then not computed), device errors. */
int mstar_integrate_adjoint(mstar_ctx *ctx, const mstar_params *params, int64_t n, const double *m, const double *x0,
                            const double *v0, double t0, double t_end, int64_t n_steps, int32_t checkpoint_every,
                            const double *gxT, const double *gvT, double gtT, double *gx0, double *gv0, double *gm,
                            mstar_stats *stats);

/* Transposed Jacobian of the accelerations applied to w [n][3] (the force
 * Hessian-vector product of the reverse kick): out_i = G sum_{j != i}
 * M(d_ij) (m_i w_j - m_j w_i), M(d) = (I - 3 d d^T / |d|^2) / |d|^3,
 * d_ij = x_j - x_i (Cartesian). */
int mstar_force_hvp(mstar_ctx *ctx, const mstar_params *params, int64_t n, const double *m, const double *x,
                    const double *w, double *out);

#ifdef __cplusplus
}
#endif
#endif /* MSTAR_H */
