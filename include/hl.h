/*
 * hl.h - C ABI of the Hermite-leapfrog wave-stepping library (libhermite_lf.so)
 *
 * The library advances the first-order acoustic system
 *
 *     p_t = -kappa div(u),     u_t = -grad(p),     kappa = c^2 constant,
 *
 * on a periodic box, or a box with reflecting walls (p = 0 on every face),
 * with the Hermite-leapfrog method of Vargas, Hagstrom, Chan and Warburton,
 * "Leapfrog time-stepping for Hermite methods" (arXiv 1808.10481):
 *   - data: value and first m derivatives per dimension at every node, scaled
 *     by h^a/a! (Sec. 2; Sec. 5 tensor-product form);
 *   - pressure on the primal grid x_j = j h at integer time levels, every
 *     velocity component on the dual grid x_{j+1/2} at half-integer levels
 *     (Sec. 2, eqs. (pGrid), (dGrid); Sec. 5);
 *   - one step = pressure half-step then velocity half-step; each builds the
 *     per-cell tensor-product Hermite-Birkhoff interpolant of degree 2m+1
 *     (Sec. 2, eq. (interp)) from the 2^d staggered neighbours and applies
 *     the odd-term leapfrog difference (Sec. 2, eq. (update1)) with
 *     Cauchy-Kowalevsky time-to-space exchange (Sec. 2, eqs. (LFloop),
 *     (final1); Sec. 3.1.2, eqs. (pdup), (vdup)).
 *
 * Conventions
 *   - Every call returns an hl_status; HL_OK == 0.  No C++ exception crosses
 *     the ABI.  On failure hl_last_error() returns a message (thread-local,
 *     valid until the next call on the same thread).
 *   - Arguments are validated on the host before anything is launched.
 *   - Device pointers (p, u, ...) are caller-owned device memory of
 *     hl_info.p_words / hl_info.u_words words of hl_info.word_bytes bytes
 *     each (hl_plan_info), in the library's device layout (below).  The caller owns the stream; a NULL
 *     stream is the default stream.  hl_step, hl_p_half and hl_u_half are
 *     asynchronous on that stream; hl_init and hl_export are synchronous.
 *   - The plan owns its operator tables and scratch; it must outlive the
 *     work enqueued with it and is freed by hl_plan_destroy.
 *
 * Host layout (hl_init input, hl_export output): FP64, C order,
 *   p[j_1]...[j_d][a_1]...[a_d],  u[i][q_1]...[q_d][a_1]...[a_d],
 * coefficient index a_k in [0, m], velocity component i in [0, d).  Primal
 * node j is at x = j h, dual node q at x = (q + 1/2) h.  Periodic: j_k and
 * q_k in [0, K_k).  Walls (the box [0, length_k] per dimension): j_k in
 * [0, K_k] (the end nodes lie on the walls), q_k in [0, K_k).
 *
 * Device layout (opaque to callers, fixed per plan): coefficient-major
 * planes, p[c][n] and u[i][c][n], with node n = i_1 + E_1 (i_2 + E_2 i_3)
 * and coefficient c = a_1 + (m+1)(a_2 + (m+1) a_3), in the plan precision.
 * Periodic: E_k = K_k for both fields.  Walls: p has E_k = K_k + 1; u is
 * padded by one ghost node per side, E_k = K_k + 2, dual node q at index
 * q + 1 (the ghosts are the mirror images of Sec. 5, "Imposing reflective
 * boundary conditions", refreshed by the library before every pressure
 * half-step)
 * (HL_FP32_COMP: hi planes p[c][n] / u[i][c][n], then the lo planes in the
 * same order).  Size limit (HL_ERR_UNSUPPORTED beyond it): one coefficient
 * plane below 4 GiB, i.e. fewer than 2^30 nodes in FP32 and FP32_COMP and
 * 2^29 in FP64.
 */
#ifndef HL_H
#define HL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HL_OK = 0,
  HL_ERR_ARG = 1,          /* invalid argument (NULL pointer, bad size, NaN) */
  HL_ERR_CFL = 2,          /* c dt / min h outside (0, 1) */
  HL_ERR_UNSUPPORTED = 3,  /* (d, m, precision) combination not built */
  HL_ERR_DEVICE = 4,       /* HIP runtime error */
  HL_ERR_NOMEM = 5,        /* host or device allocation failed */
  HL_ERR_NONFINITE = 6     /* hl_norms found a NaN or Inf */
} hl_status;

/* Storage and arithmetic type of the state.  The method is defined in exact
 * arithmetic; these are representations of its scaled nodal data (Sec. 2).
 *   HL_FP64       FP64 words, FP64 arithmetic.
 *   HL_FP32       FP32 words, FP32 arithmetic (half the bytes of FP64; the
 *                 state's rounding at every half-step is ~2^-24 relative).
 *   HL_FP32_COMP  each coefficient stored as hi + lo, hi = FP32 rounding of
 *                 the value, lo = BF16 rounding of the residual (6 bytes,
 *                 ~2^-33 relative state rounding); arithmetic in FP64.
 *                 The buffer holds every hi plane (FP32) followed by every lo
 *                 plane (BF16), counted in 2-byte words. */
typedef enum { HL_FP64 = 0, HL_FP32 = 1, HL_FP32_COMP = 2 } hl_precision;

/* Boundary of the box.
 *   HL_PERIODIC  periodic in every dimension.
 *   HL_WALLS     reflecting walls on every face: p = 0 there (Sec. 5,
 *                eq. (Boundary)), imposed by ghost dual nodes that mirror
 *                the velocity polynomials (normal component even, tangential
 *                components odd). */
typedef enum { HL_PERIODIC = 0, HL_WALLS = 1 } hl_boundary;

/* Problem statement (Sec. 4: system, CFL constant and time step; Sec. 5:
 * tensor grid with spacing h_k per dimension). */
typedef struct {
  int32_t d;            /* space dimension, 1..3 */
  int32_t m;            /* Hermite order: value + first m derivatives;
                           supported 0..7 for d = 1, 0..5 for d = 2, 0..3 for d = 3 */
  int64_t cells[3];     /* K_k >= 2 cells per dimension; entries >= d ignored */
  double  length[3];    /* period or box length per dimension, > 0; h_k = length_k / K_k */
  double  dt;           /* time step > 0, or 0 to derive dt = cfl * min_k h_k / c */
  double  cfl;          /* used when dt == 0 */
  double  c;            /* wave speed > 0; kappa = c^2 */
  int32_t precision;    /* hl_precision: storage and arithmetic type of the state */
  int32_t boundary;     /* hl_boundary */
  int32_t reserved[2];  /* must be 0 */
} hl_problem;

typedef struct {
  double  dt;           /* time step in use */
  double  nu;           /* c dt / min_k h_k, in (0, 1) */
  int64_t nodes;        /* primal nodes: prod_k K_k (periodic), prod_k (K_k + 1) (walls) */
  int32_t nc;           /* (m+1)^d coefficients per node per field */
  int32_t word_bytes;   /* 8 (FP64), 4 (FP32) or 2 (FP32_COMP) */
  int64_t p_words;      /* words of p: nc * (device p nodes), times 3 for FP32_COMP */
  int64_t u_words;      /* words of u: d * nc * (device u nodes, ghosts included), times 3 for FP32_COMP */
  int32_t tile[2];      /* tile (= workgroup) extents in x and y of the half-step launches */
  int32_t ygroup;       /* 3D: tile rows per group in the tile order (0 otherwise) */
  int32_t reserved;
} hl_info;

typedef struct hl_plan_s* hl_plan_t;

/* Build a plan: validates the problem (HL_ERR_ARG, HL_ERR_CFL when
 * c dt / min h is not in (0, 1) - the domain-of-dependence bound of
 * Sec. 3.1.1 - and HL_ERR_UNSUPPORTED), builds the interpolation operator of
 * Sec. 2 eq. (interp) exactly in rationals and the Cauchy-Kowalevsky weight
 * tables in FP64, casts them to the plan's arithmetic type and uploads them
 * to the current HIP device.  *out receives the handle (unchanged on failure). */
hl_status hl_plan(const hl_problem* prob, hl_plan_t* out);

/* Free the plan and its device tables.  NULL is accepted. */
hl_status hl_plan_destroy(hl_plan_t plan);

/* Sizes and the time step the plan uses. */
hl_status hl_plan_info(hl_plan_t plan, hl_info* out);

/* Convert host FP64 data (host layout) to the device layout and precision,
 * writing device buffers p (p_words) and u (u_words).  p0 must be non-NULL;
 * u0 == NULL means zero velocity.
 * u may be NULL (with u0 NULL and no start-up) to write p alone, e.g. the
 * data of a source for hl_add_source.
 * flags == 0:               u0 holds u at t0 + dt/2 (Sec. 2: staggered data).
 * flags & HL_INIT_STARTUP:  u0 holds u at t0; u at t0 + dt/2 is built on the
 *                           device from the odd Taylor terms over dt/2
 *                           (velocity half-step with halved weights; the
 *                           even terms of u0 are dropped, exact for u0 = 0).
 * Synchronous: returns after the data are on the device. */
#define HL_INIT_STARTUP 1u
hl_status hl_init(hl_plan_t plan, const double* p0, const double* u0, uint32_t flags,
                  void* p, void* u, void* stream);

/* Copy device state back to host FP64 arrays in host layout.  Either output
 * may be NULL to skip it.  Synchronous (waits for work on the stream). */
hl_status hl_export(hl_plan_t plan, const void* p, const void* u,
                    double* p_out, double* u_out, void* stream);

/* Advance (P^n, U^{n+1/2}) to (P^{n+nsteps}, U^{n+nsteps+1/2}) in place:
 * nsteps times a pressure half-step (Sec. 3.1.2, eq. (pdup)) followed by a
 * velocity half-step (eq. (vdup)).  nsteps >= 0.  Asynchronous.
 * For nsteps >= 16 the steps are replayed from a HIP graph of 16 steps that
 * the plan captures (on a stream of its own) for the last (p, u) pair it was
 * given; a new pair re-captures.  A plan is not safe to use from several
 * host threads at once. */
hl_status hl_step(hl_plan_t plan, void* p, void* u, int64_t nsteps, void* stream);
/* With HL_WALLS every pressure half-step (in hl_step and hl_p_half) is
 * preceded by the ghost refresh of u. */

/* One pressure half-step P <- P - sum_k w_k kappa^{k+1} Lap^k div I(U).
 * Asynchronous.  p and u must not alias.  u is not const: with HL_WALLS its
 * ghost nodes are refreshed first (its dual nodes are not changed). */
hl_status hl_p_half(hl_plan_t plan, void* p, void* u, void* stream);

/* One velocity half-step U <- U - s * sum_k w_k kappa^k grad Lap^k I(P),
 * s = weight_scale (1 for the scheme, 0.5 for the start-up).  Asynchronous. */
hl_status hl_u_half(hl_plan_t plan, void* u, const void* p, double weight_scale, void* stream);

/* Source term z(x, t) = r(t) g(x) of the pressure equation p_t = -kappa div u + z
 * (Sec. 4, eq. (waveEq1D) forcing): p += a g over every coefficient of p, with
 * g a device buffer in the p layout (written by hl_init with u = NULL from the
 * scaled Taylor data of g).  The paper does not say how z enters the step;
 * the reading taken is the midpoint rule over the step: after the pressure
 * half-step from t_n, add a = dt r(t_n + dt/2), then run the velocity
 * half-step (second order in time for the source contribution).
 * Asynchronous. */
hl_status hl_add_source(hl_plan_t plan, void* p, const void* g, double a, void* stream);

/* Variable coefficient (Sec. 4, "Smoothly varying wave speed"): kappa(x)
 * given per node as its Taylor polynomial of degree 2m+1 per variable, scaled
 * like the data: kappa~_b = prod_k h_k^{b_k} / b_k! d^b kappa (node),
 * b_k in [0, 2m+1].  kappa_p: about the primal nodes (used by the pressure
 * half-step; K+1 per dimension with HL_WALLS), kappa_u: about the dual nodes
 * (velocity half-step; K per dimension); host FP64 arrays in host layout
 * [j_1]..[j_d][b_1]..[b_d].  With HL_WALLS the ghost velocity is mirrored as
 * for constant kappa, which keeps p = 0 on the walls when kappa is even about
 * each wall.  Each half-step then runs
 * the Cauchy-Kowalevsky recurrence d_t^{2k+1} p = -(kappa Lap)^k (kappa div u),
 * d_t^{2k+1} u = -grad (kappa Lap)^k p on the cell polynomials, every product
 * truncated to degree 2m+1 per variable, k = 0..d m (where the
 * constant-coefficient series ends; the paper's variable-speed case is 1D, so
 * this length is a reading for d >= 2).  The
 * plan's c must be the largest speed (it sets the CFL check and dt).  Both
 * pointers NULL: back to the plan's constant kappa = c^2.  Built for
 * every (d, m) and precision, periodic or walls (HL_FP32_COMP keeps the kappa
 * data as hi + lo like the state); in 3D from m = 2 on, one wavefront of 64 work-items
 * updates each node (its (2m+2)^3-coefficient polynomials in LDS).
 * hl_adjoint_step then returns HL_ERR_UNSUPPORTED.  Synchronous. */
hl_status hl_set_kappa(hl_plan_t plan, const double* kappa_p, const double* kappa_u);

/* Diagnostics (off the stepping path): out[0] = sum of squares of p,
 * out[1] = sum of squares of u, accumulated in FP64 on the device; out is a
 * host array of 2 doubles.  Returns HL_ERR_NONFINITE if either is not
 * finite.  Synchronous. */
hl_status hl_norms(hl_plan_t plan, const void* p, const void* u, double* out);

/* hl_norms for callers that cannot allocate device memory (code that must
 * not call hipMalloc: tight serving loops, harnesses that forbid it): the
 * same sums, with the kernels' block partials kept in a fixed device array
 * of the library (256 blocks x at most 192 coefficient planes of FP64, 384
 * KiB, per GPU, held until the process ends) instead of the plan's buffer.
 * No call allocates (device or host).  The first call on a device looks up
 * that device's copy of the array.  Plans with more than 192 coefficient
 * planes in u (d nc > 192) get HL_ERR_UNSUPPORTED; every plan the library
 * builds fits.  Every call on a GPU shares its array: calls that overlap on
 * one GPU (several host threads) race.  Synchronous; out as for hl_norms. */
hl_status hl_norms_noalloc(hl_plan_t plan, const void* p, const void* u, double* out);

/* Discrete adjoint of hl_step: nsteps transposed steps applied in place to
 * the adjoint state (p_bar, u_bar) (device buffers laid out like p and u).
 * A step maps (P, U) to P' = P - A U, U' = U - B P'; its transpose is
 * p_bar <- p_bar - B^T u_bar, then u_bar <- u_bar - A^T p_bar (the transposed
 * half-steps in reverse order; each is a gather with the forward stencil).
 * So <step^n(x), y> = <x, adjoint^n(y)> for the plain inner product of all
 * coefficients.
 * grad_kappa == NULL: p and u are unused (may be NULL).
 * grad_kappa != NULL: a device pointer to one FP64 value, to which the
 *   derivative with respect to kappa (dt held fixed) of
 *   <p_bar, P_n> + <u_bar, U_n> (the adjoint state as passed in) is ADDED;
 *   p, u hold the forward state (P_n, U_n) after the n steps.  The library
 *   walks that state back step by step with the reversed step (half-steps
 *   with -dt in reverse order; exact in exact arithmetic) in buffers of its
 *   own, allocated on first use (p and u are not modified), and accumulates
 *   each step's contribution in FP64.
 * Reflecting walls (HL_WALLS, Sec. 5): the step is P' = P - A G U,
 * U' = U - B P' with G the ghost refresh of u (each ghost node the signed
 * mirror of an interior node), so the transpose is p_bar <- p_bar - B^T u_bar,
 * then u_bar <- u_bar - G^T A^T p_bar: A^T p_bar is formed on every slot of
 * the padded velocity array (in a plan-owned scratch array, allocated on
 * first use) and G^T adds each ghost slot, with its mirror sign, into the
 * node it mirrors.  The adjoint variables are the K dual nodes: the ghost
 * slots of u_bar are cleared first and stay zero.  The kappa gradient walks
 * the walled step back the same way (the ghost refresh of U_t before the
 * pressure-side operators read it).
 * The transposed half-steps apply dense per-corner blocks of nc x nc
 * (nc = (m+1)^d), all output rows at once up to nc = 27 and in passes of 16
 * rows beyond.  Built in every precision for every d and m (HL_FP32_COMP:
 * FP64 arithmetic on the hi + lo data, each update rounded back to hi + lo as
 * in the forward step).  Asynchronous. */
hl_status hl_adjoint_step(hl_plan_t plan, void* p_bar, void* u_bar, const void* p,
                          const void* u, void* grad_kappa, int64_t nsteps, void* stream);

/* Launch shape of the half-steps (not part of the paper: the work
 * decomposition).  Every output node is computed by one work-item with the
 * same arithmetic whatever the tile, so results do not depend on it.
 * hl_set_tile: tiles of tx x ty nodes (tx a multiple of 32 in [32, 256],
 * ty >= 1, 1 in 1D, 64 <= tx ty <= 256; tx = ty = 0: the default 64 x 4, or
 * 256 in 1D) and, in 3D, tile rows per group in the XCD-banded tile order
 * (ygroup, 0: the default 2).  hl_tune: times `reps` steps (after one warm-up
 * step) for each candidate shape (1D: 256, 128, 64; 2D/3D: 64x4, 64x2, 64x1,
 * 128x2, 128x1, 256x1, 32x8, in 3D each with y-groups 1, 2, 4) on copies of
 * (p, u) in device buffers it allocates for the call and frees, keeps the
 * fastest and reports it through hl_plan_info; p and u are not modified.  A
 * batch launches its shots with their common shape when they all have the
 * same one (read when hl_batch_step builds its descriptors), else with the
 * default.  Synchronous. */
hl_status hl_set_tile(hl_plan_t plan, int32_t tx, int32_t ty, int32_t ygroup);
hl_status hl_tune(hl_plan_t plan, const void* p, const void* u, int32_t reps, void* stream);

/* Variable-kappa adjoint (plans with hl_set_kappa; Sec. 4, "Smoothly varying
 * wave speed", differentiated): one transposed step applied in place to the
 * adjoint state (p_bar, u_bar), and the gradient of that step with respect to
 * the kappa Taylor data added to the plan's FP64 accumulators.  The step
 * being undone maps (P_t, U_t) to P' = P_t - A U_t, U' = U_t - B P'; A and B
 * depend on the kappa data (polynomially), not on the state, so the transpose
 * is p_bar <- p_bar - B^T u_bar, then u_bar <- u_bar - A^T p_bar, and the
 * accumulators receive -d<u_bar', B P'>/dkappa_u - d<p_bar, A U_t>/dkappa_p
 * (p_bar after its update, u_bar' before).  So for a loss l of the final
 * state, calling this once per step in reverse order, with the adjoint state
 * starting at dl/d(P_n, U_n), leaves dl/d(P_0, U_0) in (p_bar, u_bar) and
 * dl/dkappa in the accumulators; a loss on intermediate pressures (receivers)
 * adds its derivative to p_bar before the step that produced that pressure is
 * undone.
 * p_next: the pressure P' after the step being undone (P_{t+1});
 * u_prev: the velocity U_t before it.  Device buffers in the plan's layout,
 * not modified; the four buffers must be distinct.  Per node, the kernels run
 * the adjoint of the truncated-product recurrence (recomputing its forward
 * terms) and spread the result over the neighbouring cells with a gather (no
 * atomics), through a plan-owned scratch of d (2m+2)^d planes allocated with
 * the accumulators on first use (zeroed then).  Reflecting walls (Sec. 5):
 * the step undone is P' = P - A G U, U' = U - B P' with G the ghost refresh,
 * so u_prev's ghost layer is refreshed in a plan-owned copy before A_kappa
 * reads it, the ghost slots of u_bar are cleared and stay zero, and A^T p_bar
 * is formed on the whole padded velocity array and folded into the nodes the
 * ghosts mirror (plan-owned scratch arrays, allocated on first use).  Built
 * for d = 1 (all m), d = 2 (m <= 3) and d = 3 (m <= 1), every precision;
 * HL_ERR_UNSUPPORTED otherwise, or without kappa data.  Asynchronous. */
hl_status hl_adjoint_step_var(hl_plan_t plan, void* p_bar, void* u_bar, const void* p_next,
                              const void* u_prev, void* stream);

/* The accumulated kappa gradient: grad_p (for kappa_p) and grad_u (for
 * kappa_u), host FP64 arrays in hl_set_kappa's layout (with walls: K+1 primal
 * nodes and K dual nodes per dimension), either may be NULL.
 * reset != 0 zeroes the accumulators afterwards.  Synchronous. */
hl_status hl_kappa_grad(hl_plan_t plan, double* grad_p, double* grad_u, int reset);

/* Batched shots: many independent problems ("shots") of the same
 * d, m and precision - each with its own grid size, time step, coefficient
 * (hl_set_kappa on every plan, or on none) and buffers - advanced together,
 * one kernel launch per half-step for all of them (shot s takes its own range
 * of workgroups).  hl_batch_create keeps the plan handles (they must outlive
 * the batch).  hl_batch_step advances shot i's (p[i], u[i]) by nsteps steps,
 * exactly as hl_step on each plan would; descriptors are rebuilt (after
 * waiting for the stream) when the buffers change, and nsteps >= 16 replays a
 * captured graph of 16 batched steps.  Shots may have reflecting walls
 * (HL_WALLS): their ghost refresh is launched per shot before the batched
 * pressure half-step.  Variable kappa is batched for every d and m (3D
 * m >= 2: one workgroup per node of each shot, as in hl_step). */
typedef struct hl_batch_s* hl_batch_t;
hl_status hl_batch_create(const hl_plan_t* plans, int32_t n, hl_batch_t* out);
hl_status hl_batch_step(hl_batch_t batch, void* const* p, void* const* u, int64_t nsteps, void* stream);
hl_status hl_batch_destroy(hl_batch_t batch);

/* Sources inside the batched launch (Sec. 4: the forcing z = r(t) g(x) of the
 * pressure equation, entering each step by the midpoint rule as in
 * hl_add_source): from the next hl_batch_step on, batch step n (counted from
 * this call over every later hl_batch_step) adds amps[i][n] * g_i to shot i's
 * pressure after its pressure half-step, for n < namps.  g_i is given on the
 * primal nodes of its support: counts[i] nodes (0: no source), nodes[i][k] the
 * node's flat host index (C order over j_1..j_d, j_1 slowest), values[i] the
 * scaled Taylor data of g there, counts[i] x (m+1)^d in hl_init's coefficient
 * order.  amps[i] (namps values, NULL: zeros) are the amplitudes
 * a = dt_i r(t_n + dt_i/2) of shot i.  Host arrays, copied (values and
 * amplitudes rounded to the batch's precision; HL_FP32_COMP: the values to
 * hi + lo, as its g buffer would hold them, the amplitudes kept in FP64).
 * counts == NULL removes the sources.  Every precision; the added launch (one
 * work-item per source datum) and the step counter's update join each batched
 * step and its captured graph.  Synchronous. */
hl_status hl_batch_set_sources(hl_batch_t batch, const int64_t* counts, const int64_t* const* nodes,
                               const double* const* values, const double* const* amps, int64_t namps);

/* Message for the last failed call on this thread ("" if none). */
const char* hl_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HL_H */
