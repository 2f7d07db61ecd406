/*
 * dwos.h -- C ABI of the MI355X differential walk-on-spheres library.
 *
 * The library estimates, at chosen query points x_p inside a domain Omega(pi),
 * the solution u of the screened Poisson Dirichlet problem
 *
 *     -Lap u + sigma u = f   in Omega(pi),      u = g(., pi)   on dOmega(pi)
 *
 * (Miller et al., "Differential Walk on Spheres", TOG 43(6) 2024, Sec. 3.2,
 * eq. (bvp); the sign is chosen so that the Green's-function source term of
 * eq. (wos) enters with a plus sign), and the derivatives of u with respect
 * to every boundary parameter pi_j at once (Sec. 4, eq. (bvp_deriv); Sec. 5.1,
 * eq. (wos_deriv)), plus reverse-mode shape-functional gradients (Sec. 4,
 * eq. (functional_deriv); Sec. 5.3, eq. (ustatistics)).
 *
 * Conventions shared by every entry point
 *  - Every call returns a dwos_status; nothing throws across the ABI.  On an
 *    error the call has no effect on outputs and dwos_last_error() returns a
 *    message (thread-local, valid until the next failing call on the thread).
 *  - "host" arrays are read during the call and not retained.  "device"
 *    arrays are HIP device pointers owned by the caller; work on them is
 *    enqueued asynchronously on the stream given to dwos_create, so they must
 *    stay valid until that stream has reached the call's work.
 *  - The library copies whatever it keeps (geometry, BVH, Jacobian) into its
 *    own device allocations, released by dwos_destroy.
 *  - Sizes are element counts.  Multi-component arrays are row-major
 *    (point-major): X[p*dim + c], V[i*dim + c], udot[p*N + j].
 *  - A non-NULL dwos_stats* is host memory; filling it synchronises the stream.
 *  - Query points must lie inside Omega (the paper's eps-shell is defined
 *    inside the domain, Sec. 3.3.1); this is not checked.  A differential
 *    walk orients the boundary normal away from its last position, so a
 *    walk that starts within rounding distance of the boundary has no
 *    defined side: its offset point may fall outside the domain.
 */
#ifndef DWOS_H
#define DWOS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dwos_ctx dwos_ctx;
typedef int32_t dwos_status;

#define DWOS_OK      0
#define DWOS_EINVAL  1  /* bad argument: NULL, size, range, NaN */
#define DWOS_ENOMEM  2  /* device or host allocation failed */
#define DWOS_EDEVICE 3  /* a HIP call failed or no gfx950 device */
#define DWOS_ESTATE  4  /* call order: e.g. solve before set_boundary */

/* Working precision of the walks.  FP64 is the debug instantiation used for
 * walk-for-walk comparison with an FP64 reference. */
#define DWOS_FP32 0
#define DWOS_FP64 1

#define DWOS_MAX_LABELS 16
#define DWOS_MAX_GAUSS  8

/* Boundary data of one label (Sec. 4, "Restricted boundary data" and
 * "Mapped boundary data").
 *  kind 0 (restricted): g is the restriction of the field
 *         g(x) = c + b.x + x^T A x   (A row-major, top-left dim x dim used);
 *         the field does not depend on pi, so its parameter derivative is 0
 *         and eq. (boundary_deriv_restricted) reduces to (dg/dn - du/dn) V_n.
 *  kind 1 (mapped): per-vertex values (dwos_set_boundary's gvert) carried by
 *         the surface parameterisation and interpolated linearly over a
 *         primitive (eq. (boundary_deriv_mapped), Appendix A).  A vertex value
 *         may itself be a parameter (dwos_set_parameters' bc_pid). */
typedef struct dwos_bc {
    int32_t kind;
    int32_t pad_;
    double c;
    double b[3];
    double A[9];
} dwos_bc;

/* Problem constants (Sec. 3.2-3.3, Sec. 6.3).
 *  sigma  >= 0    screening coefficient
 *  eps    >  0    eps-shell width: a walk stops when d(x) < eps (Algorithm 1)
 *  delta  >  0    offset of the backward-difference normal derivative,
 *                 eq. (dudn_fd_estimate); delta <= eps is accepted (the
 *                 degenerate case of Sec. 6.3: the estimate is then 0)
 *  K      1..255  forward walks nested at each differential terminal (Table 1)
 *  kmax   >= 1    cap on closest-point queries per walk; the kmax-th query is
 *                 treated as terminal and counted in dwos_stats.truncated
 *  rr     0/1     Russian roulette with probability alpha = P/p^dB (Sec. 3.3)
 *  source f(x) = src_c0 + sum_i gauss[i][0] exp(-|x - m_i|^2 / (2 s_i^2)),
 *         m_i = gauss[i][1..dim], s_i = gauss[i][4]  (n_gauss <= 8)
 *  bc[l]  boundary data for primitives with label l (n_labels <= 16)
 *  dudn   0/1     normal-derivative estimator of the differential walks:
 *                 0 the backward difference (g - u(xoff))/delta of
 *                 eq. (dudn_fd_estimate); 1 the offset-point gradient
 *                 estimator of eq. (dudn_mc_estimate), the paper's ablation:
 *                 each nested walk's first step goes from xoff to
 *                 y = xoff + R s (R the largest empty ball at xoff, s
 *                 uniform) and D/R (s.n) (u(y) - g(xbar)) estimates du/dn
 *                 (g(xbar) a control variate; the paper prints 3/delta for
 *                 R = delta in 3D).  Laplace only: dudn = 1 needs sigma = 0
 *                 and no source (EINVAL), and no control variate, reflecting
 *                 or implicit boundary (ESTATE at the call). */
typedef struct dwos_problem {
    double sigma;
    double eps;
    double delta;
    int32_t K;
    int32_t kmax;
    int32_t rr;
    int32_t n_gauss;
    double src_c0;
    double gauss[DWOS_MAX_GAUSS][5];
    int32_t n_labels;
    int32_t dudn;
    dwos_bc bc[DWOS_MAX_LABELS];
} dwos_problem;

/* Counters of one call (filled when a non-NULL pointer is passed). */
typedef struct dwos_stats {
    int64_t walks;         /* forward or differential walks started */
    int64_t nested_walks;  /* forward walks nested at differential terminals */
    int64_t steps;         /* closest-point queries executed, all walks (the walk-step
                              unit); the first query of a point, shared by all its
                              walks, counts once */
    int64_t terminal;      /* main walks that reached the eps-shell */
    int64_t truncated;     /* walks cut at kmax */
    int64_t nodes;         /* BVH pair nodes visited */
    int64_t prims;         /* primitive distance tests */
    int64_t stack_overflow;/* traversals aborted for lack of stack (must be 0) */
    int64_t invalid;       /* walks ended at a non-finite position (NaN result) */
    double walk_ms;        /* device time of the walk kernel(s) of this call */
} dwos_stats;

/* Create a context for dim = 2 (polyline boundary) or 3 (triangle mesh) in
 * precision DWOS_FP32 or DWOS_FP64, enqueueing all work on `stream` (a
 * hipStream_t; NULL = the null stream).  Errors: EINVAL, ENOMEM, EDEVICE. */
dwos_status dwos_create(int32_t dim, int32_t precision, void* stream, dwos_ctx** out);

/* Release every allocation of the context (synchronises its stream). */
dwos_status dwos_destroy(dwos_ctx* ctx);

/* Message of the last failing call on this thread ("" if none). */
const char* dwos_last_error(void);

/* Boundary dOmega as nv vertices (host, nv x dim, FP64) and np primitives
 * (host, np x dim vertex indices: segments in 2D, triangles in 3D) with a
 * boundary-data label per primitive (host, np; NULL = all 0) and per-vertex
 * values for mapped labels (host, nv; NULL = 0).  Builds the BVH.
 * Primitive winding does not matter: at a closest point the normal is the
 * primitive's geometric normal oriented away from the query point, i.e. out
 * of the domain.  Errors: EINVAL (index out of range, degenerate primitive,
 * non-finite coordinate), ENOMEM. */
dwos_status dwos_set_boundary(dwos_ctx* ctx, const double* V, int64_t nv,
                              const int32_t* prims, int64_t np, const int32_t* label,
                              const double* gvert);

/* Move the vertices (device, nv x dim, FP64) keeping the topology, and refit
 * the BVH on the device (explicit surface phi(., pi), Sec. 3.1.2).
 * Errors: ESTATE without a boundary, EINVAL on NULL. */
dwos_status dwos_update_vertices(dwos_ctx* ctx, const double* V_dev);

/* Move the vertices to V(pi) = V_base + J pi for parameter values pi (device,
 * N FP64) and base positions V_base (device, nv x dim FP64), with J the
 * Jacobian of dwos_set_parameters (vertices linear in pi, as for radial or
 * Fourier displacements), then refit as dwos_update_vertices.
 * Errors: ESTATE without boundary or parameters, EINVAL on NULL. */
dwos_status dwos_apply_parameters(dwos_ctx* ctx, const double* V_base_dev, const double* pi_dev);

/* Problem constants (host struct).  Errors: EINVAL (sigma < 0, eps <= 0,
 * delta <= 0, K outside 1..255, kmax < 1, NaN, too many labels/gaussians). */
dwos_status dwos_set_problem(dwos_ctx* ctx, const dwos_problem* prob);

/* Parameters pi (N of them) as the Jacobian of the vertex positions,
 * dv_i/dpi_j, in CSR by vertex (host): rowptr[nv+1], pid[nnz] (column ids,
 * 0 <= pid < N), vel[nnz*dim].  bc_pid (host, nv, or NULL) gives, for mapped
 * labels, the parameter that a vertex's boundary value equals (-1: none).
 * The normal velocity of Sec. 3.1.2 is V_n = n . sum_k b_k dv_{i_k}/dpi_j at a
 * closest point with barycentrics b.  Errors: EINVAL, ESTATE, ENOMEM. */
dwos_status dwos_set_parameters(dwos_ctx* ctx, int64_t N, const int64_t* rowptr,
                                const int32_t* pid, const double* vel, const int32_t* bc_pid);

/* Forward solve (Algorithm 1): W walks from each of P points (device,
 * P x dim FP64).  Writes the per-point mean u_mean[P] and the variance of that
 * mean u_var[P] (device FP64; u_var may be NULL).  Walk m of point p draws
 * from the Philox4x32-10 stream keyed by `seed` with counter
 * (step, m, p, purpose | nested<<8 | instance<<16), so results do not depend
 * on launch shape.  Errors: ESTATE (no boundary/problem), EINVAL (P < 0,
 * W < 1, NULL). */
dwos_status dwos_solve(dwos_ctx* ctx, const double* X, int64_t P, int32_t W, uint64_t seed,
                       double* u_mean, double* u_var, dwos_stats* stats);

/* Allocation-free variant of dwos_solve, for callers that cannot allocate
 * device memory during the call: code under hipGraph stream capture, tight
 * serving loops, harnesses that forbid hipMalloc.  Same walks, random
 * streams and outputs as dwos_solve with the same arguments (u_mean[P],
 * u_var[P] or NULL, device FP64; X device P x dim FP64), but every workspace
 * (work-queue counter, walk counters, the per-point shared first query and
 * the per-walk values) lives in one fixed device array of 32 MiB that the
 * library holds on each device from load to process exit; the call allocates
 * and frees nothing and records no events.  Limit: the workspace must fit,
 * 1 KiB + P (4 + s) + P W s bytes with s = 4 (FP32) or 8 (FP64), each part
 * rounded up to 256 bytes: about 8.3 million walks in FP32.  Calls on one
 * device share that array and its contents persist between calls (each call
 * clears what it needs): calls that overlap in time on one device, from any
 * context or stream, race and give wrong results.  No statistics or timing.
 * Errors: EINVAL (P < 0, W < 1, NULL, workspace too small), ESTATE (no mesh
 * boundary or problem; batch, reflecting or implicit boundary). */
dwos_status dwos_solve_noalloc(dwos_ctx* ctx, const double* X, int64_t P, int32_t W, uint64_t seed,
                               double* u_mean, double* u_var);

/* Reverse mode (Sec. 4, eq. (functional_deriv), domain term): with one
 * differential walk per (p, m) (Algorithm 2, with K nested forward walks at
 * the terminal), accumulates grad[j] = sum_p w[p] * mean_m udot_m[j] into
 * grad (device, N FP64; overwritten).  w is device FP64 [P].  u_mean (device
 * [P] or NULL) receives the joint estimate of u from the same walks
 * (Sec. 5.1, observation 2).  Requires dwos_set_parameters.  Errors as
 * dwos_solve. */
dwos_status dwos_grad(dwos_ctx* ctx, const double* X, int64_t P, const double* w, int32_t W,
                      uint64_t seed, double* grad, double* u_mean, dwos_stats* stats);

/* Fused squared loss L = sum_p 1/2 (u_p - u_ref[p])^2 (Sec. 5.3): loss
 * (device, 1) gets L from the per-point walk means, grad (device, N) gets
 * sum_p [U-stat estimate of u udot - u_ref udot] using eq. (ustatistics) over
 * batches of B consecutive walks of a point, averaged over the W/B batches.
 * Errors: EINVAL unless B >= 2 and W % B == 0; otherwise as dwos_grad. */
dwos_status dwos_grad_sqloss(dwos_ctx* ctx, const double* X, int64_t P, const double* u_ref,
                             int32_t W, int32_t B, uint64_t seed, double* loss, double* grad,
                             double* u_mean, dwos_stats* stats);

/* Forward mode (Sec. 5, "forward-mode derivatives"): udot (device, P x N)
 * gets the per-point mean of udot over W differential walks, udot_var (device
 * P x N or NULL) the variance of that mean, u_mean (device P or NULL) the
 * joint u estimate.  Meant for small N (cost grows with P*N*W).
 * Errors: ENOMEM if P*N is too large for the workspace limit. */
dwos_status dwos_jvp(dwos_ctx* ctx, const double* X, int64_t P, int32_t W, uint64_t seed,
                     double* udot, double* udot_var, double* u_mean, dwos_stats* stats);

/* Sizes of the closest-point structures of a mesh boundary (host output,
 * 8 int64): [0] BVH pair nodes, [1] bytes of the node array, [2] bytes of the
 * primitive array (in the working precision, Sec. 6 layout), [3] pair nodes
 * the FP32 walk kernel stages in LDS (the breadth-first prefix), [4] 1 if it
 * stages every primitive as well, [5] primitives, [6] vertices, [7] LDS bytes
 * per block of the staged launch.  Errors: EINVAL (NULL), ESTATE (no mesh
 * boundary). */
dwos_status dwos_scene_info(dwos_ctx* ctx, int64_t* info);

/* Scheduling knobs of the walk kernels.  They change only the schedule: a
 * walk's result depends on (seed, instance, point, walk) alone, so every
 * setting gives the same walks bit for bit (the FP64 gradient sums to their
 * atomics' order).  The walks are independent (Sec. 3.3), so any order of
 * execution is valid.
 *   variant      0: one 1024-thread block per CU with the top BVH levels
 *                (and, if they fit, all primitives) staged in LDS;
 *                1: 256-thread blocks, several per CU (six wavefronts per
 *                SIMD in 3D), BVH read through the caches.  Default 1 for
 *                3D contexts, 0 for 2D.  FP64 contexts always use the
 *                unstaged kernel.
 *   park         1..64: a wavefront takes its walk step once this many of
 *                its lanes have their closest-point answer; the others
 *                resume their traversal in the next iteration (default 24)
 *   tail         0..63: a traversal round stops descending when at most this
 *                many lanes still descend while another lane holds a leaf
 *                to test; they go on in the next round (0: off; default 8)
 *   chunk        walk ids a wavefront takes from the global queue per
 *                refill: a multiple of 64 in 64..65536 (default 128)
 *   stage_nodes  cap on the breadth-first prefix of BVH nodes staged in LDS
 *                by variant 0, and on the staged prefix of the edge BVH in
 *                FP32 walk on stars over 3D reflecting meshes (-1: as many
 *                as fit; default -1) */
typedef struct dwos_tuning {
    int32_t variant;
    int32_t park;
    int32_t tail;
    int32_t chunk;
    int32_t stage_nodes;
} dwos_tuning;

/* Set or read the context's knobs (host struct).  Errors: EINVAL for a NULL
 * argument or a value out of range (the context is then unchanged). */
dwos_status dwos_set_tuning(dwos_ctx* ctx, const dwos_tuning* tuning);
dwos_status dwos_get_tuning(dwos_ctx* ctx, dwos_tuning* tuning);

#define DWOS_TUNE_CACHE 1
#define DWOS_TUNE_GRAD 2

/* Autotuner.  Times forward solves (Algorithm 1) with seed `seed` under
 * candidate knob settings by coordinate descent (variant, then park, tail,
 * chunk and, for variant 0, stage_nodes: all, a half, a quarter or none of
 * the nodes that fit; a candidate replaces the incumbent
 * when its walk-kernel time is more than 1% lower, each scored by the better
 * of two runs of the same walks) and leaves the fastest set on the context.
 * X (device) and P (host): on a single-scene context P[0] points of which
 * the first min(P[0], max(64, 2^22 / W)) are solved; on a batch context one
 * count per instance and the whole batch is solved (dwos_batch_solve).
 * flags: DWOS_TUNE_GRAD adds to each timed solve a reverse-mode call
 * (Algorithm 2: dwos_grad or dwos_batch_grad, seed + 1, unit weights, on
 * the same points) and scores the sum of both calls' walk-kernel times; it
 * needs parameters (dwos_set_parameters / dwos_batch_set_parameters).
 * DWOS_TUNE_CACHE looks the setting up in, and stores it to, a
 * process-wide table keyed by device, dimension, precision, single or batch,
 * DWOS_TUNE_GRAD and the scene's primitive count in half-octaves
 * (floor(2 log2 n)); a hit
 * applies the stored setting without running anything.  Results are stored
 * in the table in any case.  chosen (host, may be NULL) gets the setting,
 * ms (host, 2 entries, may be NULL) the walk-kernel milliseconds under the
 * setting in force at the call and under the chosen one (-1 on a cache hit).
 * Errors: as dwos_solve / dwos_batch_solve (and dwos_grad / dwos_batch_grad
 * with DWOS_TUNE_GRAD); EINVAL for unknown flags; ESTATE for DWOS_TUNE_GRAD
 * without parameters; on an error the context keeps the setting in force at
 * the call. */
dwos_status dwos_autotune(dwos_ctx* ctx, const double* X, const int64_t* P, int32_t W, uint64_t seed,
                          int32_t flags, dwos_tuning* chosen, double* ms);
/* Set only the launch shape (the variant field above). */
dwos_status dwos_set_variant(dwos_ctx* ctx, int32_t variant);

/* Graph capture.  Every hot-path call (dwos_solve, dwos_grad,
 * dwos_grad_sqloss, dwos_jvp, dwos_batch_solve, dwos_apply_parameters,
 * dwos_update_vertices) enqueues only kernels when (a) an identical call has
 * run before on the context, so workspaces and tables are in place, and (b)
 * stats is NULL; it may then be captured into a hipGraph on the context
 * stream.  Walk-kernel timing is skipped while the stream is capturing.
 * seed_dev (device, one uint64, or NULL to disable) makes every later call
 * use seed + *seed_dev, read on the device when the kernels run, so a
 * captured graph replays with fresh random streams after the caller updates
 * *seed_dev.  Errors: EINVAL on a NULL context. */
dwos_status dwos_set_seed_buffer(dwos_ctx* ctx, const uint64_t* seed_dev);

/* Per-walk records for walk-for-walk comparison.  mode 0: Algorithm 1,
 * mode 1: Algorithm 2.  u (device P*W) the walk's u estimate; steps (device
 * P*W int64 or NULL) its closest-point queries including nested walks;
 * prim (device P*W int32 or NULL) the terminal primitive or -1 when Russian
 * roulette stopped it; uoff (device P*W or NULL) the mean of the nested walks.
 * udot (device P*W*N or NULL, mode 1) the walk's full derivative vector. */
dwos_status dwos_walk_records(dwos_ctx* ctx, const double* X, int64_t P, int32_t W,
                              uint64_t seed, int32_t mode, double* u, int64_t* steps,
                              int32_t* prim, double* uoff, double* udot);

/* Closest boundary point through the BVH (Algorithm 1, DistanceToBoundary)
 * for P points (device P x dim): out (device P x 8 FP64) =
 * {d, primitive, b0, b1, b2, xbar0, xbar1, xbar2}; ties go to the lowest
 * primitive index. */
dwos_status dwos_closest(dwos_ctx* ctx, const double* X, int64_t P, double* out);

/* The ball's Green's function and Poisson-kernel scale (Sec. 3.3.1) as the
 * walk kernels evaluate them, for n (r, R) pairs (device): G|B| = G(r;R) times
 * the ball volume, and alpha = P(R)/p^dB(R).  Outputs device FP64 [n]. */
dwos_status dwos_eval_ball_kernels(dwos_ctx* ctx, const double* r, const double* R, int64_t n,
                                   double sigma, double* GB, double* alpha);

/* Accumulated device time and counters of the walk-kernel launches of one
 * kind (kind 0: forward walks, Algorithm 1; kind 1: differential walks with
 * their nested forward walks, Algorithm 2; kind 2: the adjoint walks of
 * dwos_adjoint_grad with all their nested walks) since the last reset.  Time comes
 * from events recorded on the context stream around each launch; this call
 * synchronises them.  walk_ms, launches and totals may be NULL; totals gets
 * the summed counters (walk_ms field = the same total time).
 * reset != 0 clears the accumulators of that kind after reading. */
dwos_status dwos_walk_timing(dwos_ctx* ctx, int32_t kind, int32_t reset, double* walk_ms,
                             int64_t* launches, dwos_stats* totals);

/* Memory-bandwidth probe (a measurement aid, no part of the estimator).  A
 * closest-point traversal (Algorithm 1, DistanceToBoundary) reads one BVH
 * node or primitive at an address that depends on its query, so its memory
 * roofline is the rate of random gathers of short records over the scene's
 * working set, not the streaming rate.  On the current device, with a
 * buffer of `bytes` (64 KiB .. 64 GiB, allocated and freed by the call):
 *   mode 0: random gathers of line_bytes (16, 32, 48, 64, 96 or 128) at
 *           uniformly drawn line addresses, 64 per thread, many in flight;
 *   mode 1: one coalesced streaming read of the whole buffer (line_bytes
 *           ignored).
 * The pattern is run once to warm the caches, then timed 8 times; gbps
 * (host) gets the bytes read per second of the fastest run in GB/s, ms
 * (host, may be NULL) its duration.  Errors: EINVAL, ENOMEM, EDEVICE. */
dwos_status dwos_probe_bandwidth(int64_t bytes, int32_t line_bytes, int32_t mode, double* gbps, double* ms);

/* ---- The adjoint formulation (Appendix B), an ablation ------------------
 * eq. (functional_deriv_adjoint): the derivative of a shape functional as a
 * boundary integral of the adjoint's normal derivative, the alternative to
 * the differential walks that the paper rejects because the adjoint's
 * source needs a forward walk at every step of the adjoint walk (quadratic
 * nesting).  For J = int_Omega 1/2 (u - uref)^2 with the quadratic reference
 * uref(x) = c + b.x + x^T A x (A row-major 3 x 3, the top-left dim x dim
 * used), the adjoint solves -Lap lambda + sigma lambda = u - uref in Omega,
 * lambda = 0 on the boundary (eq. (bvp_adjoint) with the operator's sign and
 * lambda flipped together), and
 *   dJ/dpi_j = int_boundary [ -dlambda/dn udot_j + l(g) V_n,j ] dsigma
 * with udot_j the boundary value of the differential problem (as at a
 * terminal of Algorithm 2, eqs. (boundary_deriv_restricted) and
 * (boundary_deriv_mapped)) and l(g) V_n,j the boundary term of
 * eq. (functional_deriv).  At each of S boundary samples y (outward normal
 * n) and for each of W walks: lambda(y - delta n) by walk on spheres with
 * zero boundary data and the source u - uref, u at each step's ball point
 * from a whole forward walk, -dlambda/dn = lambda / delta, and du/dn from K
 * forward walks from y - delta n (backward difference).
 *   grad_j = sum_s wq_s / W sum_m [ lambda_sm / delta udot_j(y_s; uoff_sm)
 *                                   + 1/2 (g(y_s) - uref(y_s))^2 V_n,j(y_s) ]
 * code (device int32 [S]): primitive * 2 + flip, flip = 1 when the outward
 * normal is minus the primitive's geometric normal ((b - a) turned clockwise
 * for a segment a->b, (b - a) x (c - a) for a triangle); bary (device FP64
 * S x (dim - 1)): barycentrics b1 (, b2) of the vertices 1 (, 2), vertex 0
 * taking the rest; wq (device FP64 [S]): quadrature weights (|boundary| / S
 * for uniform samples).  grad (device FP64 [N]) is overwritten.  rec_lambda
 * and rec_uoff (device FP64 S x W, may be NULL) receive lambda_sm and the
 * offset means uoff_sm.  Walk m of sample s draws Philox4x32-10 counters
 * (k, m, s, 0x10) for adjoint step k (0x12: a 3D step's second draw),
 * (k, m, s, 0x20 | k' << 8) for the forward walk at adjoint step k', and
 * (k, m, s, 0x30 | i << 8) for the i-th offset walk.  Samples on a primitive
 * that moves with no parameter run no walks (lambda 0, uoff = g).
 * Errors: EINVAL (NULL or bad arguments, a code naming no primitive, more
 * than 2^30 walks); ESTATE (no boundary, problem or parameters, a batch
 * context, an implicit or reflecting boundary, an attached control variate,
 * dudn != 0). */
typedef struct dwos_quad {
    double c;
    double b[3];
    double A[9];
} dwos_quad;
dwos_status dwos_adjoint_grad(dwos_ctx* ctx, const int32_t* code, const double* bary, const double* wq,
                              int64_t S, const dwos_quad* uref, int32_t W, uint64_t seed, double* grad,
                              double* rec_lambda, double* rec_uoff, dwos_stats* stats);

/* ---- Batched instances: many boundaries and query sets in one launch ----
 * A batch context holds I instances, each with its own boundary, BVH, sigma,
 * eps, delta and query points; all instances share the other problem
 * constants and the boundary-data table.  Walk m of point p of instance i
 * uses the Philox counter (step, m, p, purpose | nested<<8 | i<<16). */

/* Append an instance (same arguments as dwos_set_boundary plus its own
 * screening and shell constants).  Must be called before dwos_batch_solve;
 * the instance index is written to *index.  Errors: EINVAL, ENOMEM. */
dwos_status dwos_batch_add_instance(dwos_ctx* ctx, const double* V, int64_t nv,
                                    const int32_t* prims, int64_t np, const int32_t* label,
                                    double sigma, double eps, double delta, int32_t* index);

/* Parameter Jacobian of instance `index` (host arrays over that instance's
 * own vertices, laid out as dwos_set_parameters' rowptr / pid / vel; N = 0
 * clears it).  In dwos_batch_grad the parameters of instance i come after
 * those of instances 0..i-1.  Errors: EINVAL (no such instance, bad N,
 * rowptr, pid or velocity). */
dwos_status dwos_batch_set_parameters(dwos_ctx* ctx, int32_t index, int64_t N, const int64_t* rowptr,
                                      const int32_t* pid, const double* vel);

/* Reverse mode over every instance in one persistent launch (Algorithm 2
 * with each instance's constants, Sec. 5.3's weighted sum): grad (device,
 * sum_i N_i FP64) = sum_p w_p udot(x_p) over all instances' points, X_all
 * and w (device) back to back as in dwos_batch_solve, P (host) the counts;
 * u_mean (device, sum_i P[i], or NULL) the joint u estimates.  Every instance
 * must share delta (the offset of the normal derivative).
 * Errors: EINVAL (counts, NULL arguments, differing delta, an instance with
 * sigma > 0 while the problem's rr = 0), ESTATE (no
 * instances, problem or parameters; control variate or gradient normal-
 * derivative estimator set), ENOMEM (more than 2^28 walks). */
dwos_status dwos_batch_grad(dwos_ctx* ctx, const double* X_all, const int64_t* P, const double* w,
                            int32_t W, uint64_t seed, double* grad, double* u_mean, dwos_stats* stats);

/* Solve every instance in one persistent launch: X_all (device) holds the
 * instances' points back to back (sum_i P[i] x dim), P (host, I counts),
 * W walks per point; u_mean/u_var (device, sum_i P[i]).  Errors as solve;
 * EINVAL also for an instance with sigma > 0 while the problem's rr = 0
 * (screening needs Russian roulette, Sec. 3.3). */
dwos_status dwos_batch_solve(dwos_ctx* ctx, const double* X_all, const int64_t* P,
                             int32_t W, uint64_t seed, double* u_mean, double* u_var,
                             dwos_stats* stats);

/* ---- Learned control variate of the nested walks ----
 * An extension of the method: the paper lists variance reduction and caches
 * that estimate u without a walk as future work (Sec. 8; Appendix B).
 *
 * A network N(x): features [sin 2 pi B x, cos 2 pi B x, x, 0...] (64 inputs;
 * B is F x dim, 2F + dim <= 64), four tanh layers of width 64 and a linear
 * scalar output; parameters theta (dwos_mlp_theta_size() FP32 values, for
 * l = 1..4: W_l 64 x 64 row-major with row = output unit, then b_l; then
 * w_5[64], b_5).  The products run on the matrix cores with split-BF16
 * operands (hi + lo, about 16 mantissa bits) and FP32 accumulation.
 *
 * For any smooth N, the ball's mean-value identity of the screened operator
 * (Sec. 3.3) applied at each step of a nested walk (Algorithm 1) makes
 *   C = N(x_0) - sum_j |B_j| G_j (-Lap N + sigma N)(y_j) - [alive] N(x_stop)
 * a zero-mean quantity ("alive": the walk ended in the eps-shell or at the
 * cap, not by roulette).  With a network attached, each differential
 * terminal (Algorithm 2) estimates u(xoff) by
 *   N(xoff) + [run] (uhat + C_mean) / q
 * where the K nested walks run with probability q (a Philox draw of the
 * terminal step, counter purpose 4), the source-step sum is estimated by one
 * step chosen uniformly along the walk (reservoir sampling, counter purpose
 * 4 of each nested step) weighted by the number of source steps, and C_mean
 * averages C over the K nested walks.  The mean is that of the plain
 * estimator for any N and q; the variance vanishes as N approaches u.  The
 * walks themselves (and their random numbers) are unchanged.
 * C enters with a coefficient beta (N(xoff) and C_mean scaled by beta):
 * 1 on the first call after attaching, then the variance-minimising
 * -E[uhat C] / E[C^2] estimated on the device from the previous call's walks
 * and clamped to [0, 1], so it never depends on the walks it weights. */
typedef struct dwos_mlp dwos_mlp;

int32_t dwos_mlp_theta_size(void);

/* Create a network with frequencies B (host, F x dim FP32) on the current
 * device, work enqueued on `stream` (hipStream_t, NULL = null stream).
 * theta starts at zero (N = 0); the Adam moments at zero.
 * Errors: EINVAL (dim, F, NULL or non-finite B), ENOMEM, EDEVICE. */
dwos_status dwos_mlp_create(int32_t dim, int32_t F, const float* B, void* stream, dwos_mlp** out);
void dwos_mlp_destroy(dwos_mlp* m);

/* Copy theta in (device, FP32) and reset the Adam state / out (device). */
dwos_status dwos_mlp_set_params(dwos_mlp* m, const float* theta);
dwos_status dwos_mlp_get_params(dwos_mlp* m, float* theta);

/* N at n points X (device, n x dim FP32) into N (device n); if grad (device
 * n x dim) or lap (device n) is non-NULL, also grad N and Lap N (value,
 * gradient and Laplacian channels carried through every layer). */
dwos_status dwos_mlp_eval(dwos_mlp* m, const float* X, int64_t n, float* N, float* grad, float* lap);

/* Gradient of the training loss sum_i 1/2 w_i (N(x_i) - t_i)^2 (w device or
 * NULL for all 1) into the network's gradient buffer; loss (device, one
 * float, may be NULL) gets the loss and grad (device, theta size, may be
 * NULL) a copy of the gradient. */
dwos_status dwos_mlp_loss_grad(dwos_mlp* m, const float* X, const float* T, const float* w, int64_t n,
                               float* loss, float* grad);

/* Gradient of sum_i (Nbar_i N(x_i) + Lbar_i Lap N(x_i)) (Nbar, Lbar device
 * n floats; Lbar may be NULL) into the network's gradient buffer; grad
 * (device, may be NULL) gets a copy.  The Laplacian's parameter derivative is
 * carried by reverse mode through the value, gradient and Laplacian
 * channels of every layer. */
dwos_status dwos_mlp_vjp(dwos_mlp* m, const float* X, const float* Nbar, const float* Lbar, int64_t n,
                         float* grad);

/* One Adam step (Kingma and Ba 2015) with the last computed gradient. */
dwos_status dwos_mlp_adam_step(dwos_mlp* m, float lr, float beta1, float beta2, float eps);

/* Attach a network (not owned; NULL detaches) with nested-walk probability
 * q in (0, 1] to a context: every later differential call (dwos_grad,
 * dwos_grad_sqloss, dwos_jvp, dwos_walk_records mode 1) uses the control
 * variate.  Errors: EINVAL (q, dimension or device mismatch). */
dwos_status dwos_cv_attach(dwos_ctx* ctx, dwos_mlp* m, double q);

/* The coefficient beta the next differential call will use (host output;
 * synchronises the context stream).  Errors: EINVAL, ESTATE (no network). */
dwos_status dwos_cv_beta(dwos_ctx* ctx, double* beta);

/* Train the attached network for `steps` Adam steps (lr; beta 0.9, 0.999;
 * eps 1e-8) on the records of the last differential chunk.  The objective is
 * the sample variance of the control-variate estimate: since E[C] = 0,
 * E[(uhat + C)^2] = Var(uhat + C) + u^2, so each step draws `batch` walks
 * (Philox key seed) and minimises the mean of (uhat + C)^2/2 (through N at
 * the offset and stop points and N, Lap N at the ball samples) plus
 * (N(xbar) - g(xbar))^2/2 at their terminal points (N(xoff) serves as a
 * baseline held fixed in the differentiation).  loss (device, one
 * float, may be NULL) gets the last step's objective.  Records are consumed
 * after they were used, so a network never corrects the walks it was
 * trained on.  Errors: ESTATE (no network or no records), EINVAL. */
dwos_status dwos_cv_train(dwos_ctx* ctx, int32_t steps, int32_t batch, float lr, uint64_t seed,
                          float* loss);

/* Differential walks with the control variate, exported per walk (device
 * P*W*9 FP64: run (-1 no terminal, 0 skipped, 1 run), xoff[3], plain nested
 * mean, control-variate estimate, training target, u, terminal primitive)
 * and per nested walk (device P*W*K*10: L, alive, xstop[3], y[3], rho, d).
 * Errors: as dwos_walk_records; ESTATE without an attached network. */
dwos_status dwos_cv_walk_records(dwos_ctx* ctx, const double* X, int64_t P, int32_t W, uint64_t seed,
                                 double* walk, double* nested);

/* ---------------------------------------------------------------------------
 * Reflecting boundaries: walk on stars.
 *
 * The mixed problem of Sec. 3.4, eq. (mixed_bvp): the Neumann or Robin
 * condition (dwos_set_robin; zero flux by default) on a fixed part of the
 * boundary that does not depend on the parameters, the Dirichlet data g
 * elsewhere.  Its parameter derivative (Sec. 4.4, eq. (mixed_bvp_deriv))
 * nests through the Dirichlet boundary only.  The paper takes the estimator
 * from the walk-on-stars papers it cites; each step uses the star radius
 * R = min(distance to the Dirichlet boundary, distance to the closest
 * silhouette point of the reflecting boundary -- a vertex of the 2D
 * polyline, an edge of the 3D triangle mesh --, at least 16 units of
 * rounding of the position), a uniform direction (at a reflecting boundary
 * point: uniform over the directions entering the domain), and the first
 * reflecting point hit along it before R as the next point, weighted by the
 * ratio of the ball's Poisson kernel there to the direction density
 * (dwos_eval_reflect_weight); the source is sampled along the same
 * direction and counted inside the visible region.  One Philox draw per
 * step: word 0 (2D) or words 0 and 1 (3D) the direction, word 2 the
 * roulette, word 3 the source radius.  Every solve / grad / jvp / records
 * call then runs walks on stars; the control variate and batch contexts are
 * not available with a reflecting boundary (ESTATE).
 * ------------------------------------------------------------------------- */

/* Reflecting boundary as ns primitives (host, ns x dim vertex indices) over
 * nv vertices (host, nv x dim, FP64) of its own; ns = 0 removes it.
 * 2D: segments, each with the domain on its left (from its first to its
 * second vertex): closed outer walls counter-clockwise, obstacles clockwise.
 * Segments meeting at a shared vertex index are adjacent; a vertex with one
 * segment (an open end) or with more than two always counts as a
 * silhouette.  Builds a BVH over the segments.
 * 3D: triangles a, b, c, each with the domain on the side its left normal
 * (b - a) x (c - a) points to.  Triangles sharing two vertex indices share
 * an edge; seen from x an edge of two triangles is a silhouette when both
 * lie on the same side of the plane through x and the edge, and an edge of
 * one triangle (a rim) or of more than two always is.  Builds a BVH over the
 * triangles (ray hits, Robin samples) and one over the edges (silhouettes).
 * The walls are one-way: a walk meets a wall only from its domain side, so
 * a walk that rounding puts just behind a wall passes back into the domain
 * (in exact arithmetic this is the same as taking the side a walk arrives
 * from).  Errors: EINVAL (index out of range, zero-length segment or
 * zero-area triangle, non-finite coordinate, more than 65536 primitives with
 * a Robin condition set), ESTATE (batch or implicit-boundary context),
 * ENOMEM. */
dwos_status dwos_set_reflecting(dwos_ctx* ctx, const double* V, int64_t nv, const int32_t* segs, int64_t ns);

/* Robin condition on the reflecting boundary (Sec. 3.4, eq. (mixed_bvp)):
 *   du/dn - mu u = h    with n the unit normal pointing into the domain,
 * mu >= 0 a constant and h (host struct, NULL: h = 0) a restricted field
 * h(x) = c + b.x + x^T A x (kind 0; A row-major 3 x 3, the top-left
 * dim x dim used).  mu = 0 and h = NULL restore the zero-flux boundary.  Neither may
 * depend on the parameters.  The differential walks (Sec. 4.4,
 * eq. (mixed_bvp_deriv)) keep mu with zero data and nest through the
 * Dirichlet boundary only.  Each walk-on-stars step then also estimates the
 * boundary terms -int G (mu u + h) of the star-shaped region's integral
 * equation over the reflecting boundary inside its ball.  2D: a point z
 * uniform by length there (the segment chosen by an exponential race in
 * which reflecting segment o draws Philox counter (k, m, p, tag | 8 |
 * o << 16) and weighs in with its clipped length; L the reflecting length in
 * the ball; word 1 of the step's draw decides the branch below).  3D: the
 * triangles that reach into the ball with their whole areas (L their sum),
 * the same race with areas as weights, z uniform on the winner (words 1 and
 * 2 of its draw) and counted only inside the ball; word 3 of the winner's
 * draw decides the branch.  The data term is added directly and the mu term
 * by continuing the walk at z with probability q = min(1/2, c mu L G) (c = 2
 * on a wall, 1 inside), with the walk's throughput carrying the weights'
 * signs and sizes; with mu > 0 the star radius is also capped at 1/mu.
 * Errors: EINVAL (mu < 0 or not finite, h not kind 0 or not finite, more
 * than 65536 reflecting primitives), ESTATE (no reflecting boundary when
 * mu > 0 or h != NULL). */
dwos_status dwos_set_robin(dwos_ctx* ctx, double mu, const dwos_bc* h);

/* Query points that lie on the reflecting boundary (host, P entries: the
 * reflecting primitive a point lies on -- its domain side being the
 * primitive's left, as for dwos_set_reflecting --, or -1 for a point
 * inside).  Applies
 * to every later call, which must then have exactly P points; seg = NULL or
 * P = 0 clears it.  Errors: EINVAL (index out of range), ESTATE (no
 * reflecting boundary). */
dwos_status dwos_set_start_segments(dwos_ctx* ctx, const int32_t* seg, int64_t P);

/* The two reflecting-boundary queries of a walk-on-stars step at n rows
 * (device arrays, dim = the context's dimension): X (n x dim), dir (n x dim,
 * unit), cap (n), on (n, int32: primitive the point lies on or -1), nin
 * (n x dim: domain side when on >= 0).  out (n x 3): distance to the
 * closest silhouette point (vertex in 2D, edge in 3D; capped at cap), t of
 * the first reflecting primitive entered from its domain side by X + t dir
 * with 0 <= t < cap (cap if none), that primitive or -1.  A row with an
 * invalid `on` gets NaN.  Errors: ESTATE (no reflecting boundary), EINVAL. */
dwos_status dwos_reflect_query(dwos_ctx* ctx, const double* X, const double* dir, const double* cap,
                               const int32_t* on, const double* nin, int64_t n, double* out);

/* Step weight at a reflecting boundary point at distance r inside the ball
 * of radius R (device arrays of n): |dS_1| r^(dim-1) |dG/dr|(r; R) with G
 * the ball's Green's function, i.e. k r [K1(kr) + K0(kR) I1(kr)/I0(kR)]
 * (2D) or [kr cosh(k(R-r)) + sinh(k(R-r))]/sinh(kR) (3D), k = sqrt(sigma),
 * in the context's working precision.  Errors: EINVAL. */
dwos_status dwos_eval_reflect_weight(dwos_ctx* ctx, const double* r, const double* R, int64_t n,
                                     double sigma, double* w);

/* ---------------------------------------------------------------------------
 * Implicit boundaries from harmonic monopoles (2D; Sec. 7.4, "Image-space
 * curve inflation").  The boundary is the zero set of
 *   h(x) = c + sum_n a_n / |x - p_n|,   c < 0, every a_n > 0,
 * and the domain is {h > 0} (the points nearer the monopoles).  The
 * parameters are pi = (a_0, p_0x, p_0y, a_1, ...) (N = 3n), and their
 * normal velocity is the level-set one of Sec. 3.1,
 * eq. (normal_velocity): V_n = (dh/dpi) / |grad h|.
 * Each step of Algorithm 1 and Algorithm 2 takes a safe disk instead of the
 * largest empty one: the larger of the Harnack radius of h - c (a positive
 * harmonic function of 3D space, with the poles at the p_n) and the radius
 * at which sum_n a_n / (|x - p_n| + d) falls to -c.  A walk stops when
 * h <= |grad h| eps where h < -c (the gradient-sensitive shell; the second
 * condition keeps the test from firing next to a pole), and takes the
 * boundary value at the Newton projection xbar = x - h grad h / |grad h|^2.
 * The boundary data are the restricted data of label 0 (dwos_set_problem,
 * kind 0); the outward normal at xbar is -grad h / |grad h|.  The random
 * numbers and step order are those of the walk-on-spheres kernel.
 * Every solve / grad / grad_sqloss / jvp / walk_records call then walks on
 * the implicit boundary and differentiates with respect to the 3n monopole
 * parameters (dwos_set_parameters is not used).  A context holds either a
 * mesh boundary or an implicit one; reflecting boundaries, the control
 * variate and batch contexts are not available with it (ESTATE).  A walk
 * that lands exactly on a monopole's position (where h is not defined) ends
 * with a NaN result and counts as invalid in dwos_stats.
 * ------------------------------------------------------------------------- */

/* Implicit boundary of n monopoles (host, n x 3 FP64: a_n, p_nx, p_ny) and
 * the constant c; n = 0 removes it.  The table is copied (converted to the
 * working precision); the call returns once the copy is done.
 * Errors: EINVAL (3D context, n > 1024, a_n <= 0, c >= 0, non-finite
 * values), ESTATE (mesh or reflecting boundary, attached control variate,
 * batch context), ENOMEM. */
dwos_status dwos_set_implicit(dwos_ctx* ctx, const double* mono, int64_t n, double c);

/* The band term of the shape-functional derivative on an implicit boundary
 * (Sec. 7.4, "Implicit boundary integrals"): the boundary integral of
 * eq. (functional_deriv) taken as a volume integral over the band of the
 * domain next to the boundary.  For every point x_p (device, P x 2 FP64)
 * in the band, adds coef_p V_n(x_p) to grad (device, 3n FP64, accumulated,
 * not cleared):
 *   grad_j += coef_p (dh/dpi_j)(x_p) / |grad h(x_p)|.
 * The band is h > 0, h < eps_band |grad h| and h < -c, i.e. the first-order
 * distance h / |grad h| to the zero set is below eps_band (away from the
 * poles).  The caller folds its quadrature weight, the loss at x_p and the
 * band normalisation into coef (device, P FP64).  region (device, P int32)
 * receives, if non-null, 1 for the points in the band, 2 for the other
 * points of the domain (h > 0) and 0 for the points outside, so that the
 * domain term can take the points labelled 2.
 * Errors: EINVAL (bad arguments, eps_band <= 0), ESTATE (no implicit
 * boundary). */
dwos_status dwos_implicit_band_grad(dwos_ctx* ctx, const double* X, int64_t P, const double* coef,
                                    double eps_band, double* grad, int32_t* region);

/* ---------------------------------------------------------------------------
 * Remeshing (host code): the periodic isotropic remeshing of the paper's
 * shape-optimisation loop (Sec. 7.2, "Gradient preconditioning", after
 * Botsch and Kobbelt).  Each of `iters` iterations splits edges longer than
 * 4L/3, collapses edges shorter than 4L/5 (never creating an edge longer
 * than 4L/3, changing the topology or flipping a triangle), flips edges
 * toward valence 6 (3D), moves free vertices to their neighbours' centroid
 * within the tangent plane (line) and projects them back onto the input.
 * ------------------------------------------------------------------------- */
typedef struct dwos_mesh dwos_mesh;

/* Remesh a boundary: dim 2 (polylines: every vertex has at most one
 * segment in and one out; open ends stay) or 3 (triangles: no edge in more
 * than two; vertices on border edges stay), V host nv x dim FP64, prims host
 * np x dim, fixed host nv int32 or NULL (nonzero: the vertex neither moves
 * nor disappears, and an edge between two fixed vertices is neither split
 * nor collapsed), target edge length L > 0, iters in 0..100.  The result
 * is owned by *out (dwos_mesh_destroy); orientation is preserved.  Runs on
 * the host only (no device or stream is touched).
 * Errors: EINVAL (bad dim, empty mesh, index out of range, degenerate
 * primitive, non-finite coordinate, L <= 0, non-manifold input). */
dwos_status dwos_remesh(int32_t dim, const double* V, int64_t nv, const int32_t* prims, int64_t np,
                        const int32_t* fixed, double target, int32_t iters, dwos_mesh** out);

/* Vertex and primitive counts of a remeshed boundary. */
dwos_status dwos_mesh_size(const dwos_mesh* m, int64_t* nv, int64_t* np);

/* Copy out (host buffers sized by dwos_mesh_size; any may be NULL) the
 * vertices (nv x dim), primitives (np x dim) and, per vertex, the index of
 * the input vertex it continues, or -1 for a vertex a split created. */
dwos_status dwos_mesh_get(const dwos_mesh* m, double* V, int32_t* prims, int64_t* src);

/* Release a remeshed boundary (NULL is ignored). */
void dwos_mesh_destroy(dwos_mesh* m);

/* ---------------------------------------------------------------------------
 * Shape-optimisation step for mesh vertices (the optimiser of the paper's
 * experiments, Sec. 6 "Implementation and evaluation" and Sec. 7.2
 * "Gradient preconditioning"): vector Adam (second moment per vertex from
 * the squared norm of its gradient) on u = (I + lambda L) x, L the
 * combinatorial Laplacian of the mesh over edges between movable vertices,
 * with the step size set by the largest second moment over the movable
 * vertices:
 *   g_u = M^-1 g_x,  m = b1 m + (1-b1) g_u,  v_i = b2 v_i + (1-b2)|g_u,i|^2,
 *   u -= lr m_hat / (sqrt(max_i v_hat_i) + eps),  x = M^-1 u,
 * M = I + lambda L.  The solves are Jacobi-preconditioned conjugate
 * gradients on the device, warm-started from the previous solution and
 * stopped when the preconditioned residual norm falls below tol times its
 * starting value (or after max_iters).  Device arrays x and g are nv x dim,
 * row-major; calls are asynchronous on the stream given at creation except
 * for one small device-to-host read of a convergence flag every 16
 * iterations.
 * ------------------------------------------------------------------------- */
typedef struct dwos_opt dwos_opt;

/* Build M from the primitives (host, np x dim vertex indices: segments or
 * triangles) over nv vertices; movable (host, nv, nonzero = movable; NULL:
 * all) marks the vertices the optimiser may move (a fixed vertex keeps its
 * position and its row of M is the identity); lambda >= 0.
 * Errors: EINVAL, ENOMEM, EDEVICE. */
dwos_status dwos_opt_create(int32_t dim, int64_t nv, const int32_t* prims, int64_t np, const int32_t* movable,
                            double lambda, void* stream, dwos_opt** out);
void dwos_opt_destroy(dwos_opt* opt);

/* Start from vertex positions x (device): u = M x, zero moments. */
dwos_status dwos_opt_reset(dwos_opt* opt, const double* x);

/* One step with the gradient g = dJ/dx (device); x (device) is updated in
 * place.  iters (host, 2, may be NULL): CG iterations of the two solves.
 * Errors: EINVAL, ESTATE (no reset). */
dwos_status dwos_opt_step(dwos_opt* opt, const double* g, double* x, double lr, double beta1, double beta2,
                          double eps, int32_t max_iters, double tol, int32_t* iters);

/* x := M^-1 b (device arrays), starting from the x given.  iters (host):
 * CG iterations used. */
dwos_status dwos_opt_solve(dwos_opt* opt, const double* b, double* x, int32_t max_iters, double tol,
                           int32_t* iters);

#ifdef __cplusplus
}
#endif

#endif /* DWOS_H */
