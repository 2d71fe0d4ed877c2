/*
 * libjgs2 -- C ABI of the MI355X (gfx950) JGS2 per-iteration solver.
 *
 * Method: Lan et al., "JGS2: Near Second-order Converging Jacobi/Gauss-Seidel
 * for GPU Elastodynamics" (arXiv 2506.06494).  Each implicit-Euler step
 * minimises the incremental potential E = I + Psi (Sec. 3, Eq. variation) by
 * parallel per-vertex 3x3 Newton sweeps (Sec. 8.1), optionally corrected by
 * the precomputed co-rotated, cubature-sampled subspace of Secs. 4-6
 * (Eqs. tilde_phi, reduced_local, reduced_h_g, cubature, u).
 *
 * Conventions shared by every entry point:
 *   - Every function returns an int32 status (JGS2_OK or a negative code);
 *     no exception crosses the ABI.  jgs2_last_error() describes the last
 *     failure of a handle.
 *   - Host arrays are read or written during the call only and never
 *     retained.  Arrays of vertices are row-major (nV x 3), arrays of tets are
 *     row-major (nT x 4) of vertex ids.
 *   - The library owns all device memory it allocates and frees it in
 *     jgs2_destroy().  Work is ordered on the handle's HIP stream (the null
 *     stream unless jgs2_set_stream() was called); calls that return host
 *     data synchronise that stream.
 *   - A handle is not thread-safe: use one handle per host thread / stream.
 */
#ifndef JGS2_H
#define JGS2_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes.  JGS2_NOT_CONVERGED is positive: the call completed and
 * kept its results, but a solve stopped at its sweep cap above its
 * tolerance; the negative codes are failures. */
#define JGS2_NOT_CONVERGED 1
#define JGS2_OK            0
#define JGS2_E_INVALID    -1  /* bad argument, size, order of calls, non-finite input */
#define JGS2_E_OOM        -2  /* device allocation failed */
#define JGS2_E_HIP        -3  /* a HIP runtime call failed */
#define JGS2_E_NOT_READY  -4  /* mesh, material, correction or state missing */
#define JGS2_E_DIVERGED   -5  /* residual grew past 1e8 x its start value */
#define JGS2_E_INFEASIBLE -6  /* a vertex is on or behind a contact plane */
#define JGS2_E_NONFINITE  -7  /* NaN/Inf appeared in the residual */
#define JGS2_E_BOUNDS     -8  /* bounds-checked build: an index check in a sweep kernel failed */

/* Local system of a vertex sub-problem (Sec. 8.1: one sub-problem per vertex,
 * N_i = 3).
 *   JGS2_PLAIN    A_i = H_ii (assembled diagonal block), b_i = g_i: the plain
 *                 per-vertex Newton relaxation without overshoot correction.
 *   JGS2_CUBATURE A_i, b_i from the co-rotated subspace Phi_{i,a} =
 *                 R_a Ubar_{i,a} R_i^T (Eq. tilde_phi): incident elements and
 *                 one-ring gradients exactly, remote elements by the
 *                 cubature samples of Eq. cubature (reading R3, see the
 *                 design notes).
 *   JGS2_DAMPER   A_i = H_ii + sum_s w_s Phi_s^T H_s Phi_s over the cubature
 *                 samples (the sampled reduced Hessian of Eq. cubature as a
 *                 damper on the local solve, Sec. 5's closing remark),
 *                 b_i = g_i (the sampled gradient left out).  Uses the same
 *                 correction tables as JGS2_CUBATURE.
 *   JGS2_EXACT    the exact co-rotated subspace in the literal form of
 *                 Eq. local_newton, with Eq. relation's derivatives of E_C:
 *                 A_i = H_ii + sum_{a in N(i)} H_{i,a} Phi_{i,a} (the one
 *                 ring; symmetrised), b_i = sum_a Phi_{i,a}^T g_a over every
 *                 free vertex (no cubature).  At rest a Jacobi sweep is the
 *                 Newton step (Sec. 4.2).  Since U-bar_{i,a} =
 *                 (H-bar^-1)_{a,i} B_i^-1 (Eq. u), jgs2_precompute keeps the
 *                 symmetric H-bar^-1 once on the device (about nVf^2 x 18
 *                 bytes in FP32) and b_i = R_i B_i^-1 (H-bar^-1 h)_i with
 *                 h_a = R_a^T g_a.                                            */
#define JGS2_PLAIN     0
#define JGS2_CUBATURE  3
#define JGS2_DAMPER    4
#define JGS2_EXACT     5

/* Parallel order (Sec. 8.1): Jacobi (all vertices from one iterate) or
 * coloured Gauss-Seidel (greedy colours in ascending order; gradients and
 * rotations refreshed before each colour). */
#define JGS2_JACOBI    0
#define JGS2_GS        1

#define JGS2_MAX_PLANES 8

typedef struct jgs2_solver jgs2_solver;

typedef struct jgs2_params {
    double  dt;                 /* time step h [s] */
    double  gravity[3];         /* f_ext / m [m/s^2] */
    int32_t variant;            /* JGS2_PLAIN, JGS2_CUBATURE, JGS2_DAMPER or JGS2_EXACT */
    int32_t order;              /* JGS2_JACOBI or JGS2_GS */
    double  omega;              /* step scale: x_i += omega dx_i (1 = none) */
    double  rel_tol;            /* stop when |g| / |g(x0)| <= rel_tol */
    int32_t max_sweeps;         /* sweep cap per step */
    int32_t check_every;        /* sweeps between residual reads (>= 1) */
    double  d_hat;              /* IPC barrier activation distance (Eq. barrier) */
    double  kappa;              /* barrier stiffness (not given in the paper) */
    int32_t n_planes;           /* static planes n . x >= c, 0..JGS2_MAX_PLANES */
    int32_t line_search;        /* 1: feasibility clamp + energy backtracking */
    double  planes[JGS2_MAX_PLANES][4];  /* (n_x, n_y, n_z, c), n unit length */
    double  adj_rel_tol;        /* adjoint solves stop at |H y - b| / |b| <= adj_rel_tol */
    int32_t adj_max_sweeps;     /* sweep cap per adjoint solve */
    int32_t use_graph;          /* 1: replay each group of check_every sweeps and its
                                   residual check as one captured HIP graph */
    double  exact_drop;         /* JGS2_EXACT: tiles of H-bar^-1 whose largest entry is at
                                   most exact_drop x the largest entry of H-bar^-1 are
                                   skipped by the sweep (0 keeps every tile; default
                                   1e-10, at the FP32 resolution of the product); may
                                   change between steps without a new precompute */
} jgs2_params;

typedef struct jgs2_step_stats {
    int32_t sweeps;             /* sweeps performed this step (the most of any body) */
    int32_t status;             /* JGS2_OK, JGS2_NOT_CONVERGED, JGS2_E_DIVERGED, ... */
    double  r0;                 /* |g(x0)| over free DOFs */
    double  r_final;            /* largest |g_b(x)| / |g_b(x0)| over bodies at the end */
    double  seconds;            /* device time of the step (HIP events) */
    int32_t ls_halvings;        /* energy backtracking halvings this step */
    int32_t reserved;
    double  dx_norm;            /* |x_k - x_{k-1}| over free DOFs of the last sweep [m]
                                   (the convergence measure of Sec. 8 / Table 1) */
} jgs2_step_stats;

typedef struct jgs2_adjoint_stats {
    int32_t steps;              /* steps pulled back */
    int32_t status;             /* JGS2_OK or the first failure */
    int64_t adjoint_sweeps;     /* linear sweeps over all steps */
    int64_t forward_sweeps;     /* sweeps of the recomputed forward steps */
    double  max_rel_res;        /* largest final |H y - b| / |b| over the steps */
    double  seconds;            /* device time of the whole backward pass */
} jgs2_adjoint_stats;

/* Fills *p with defaults: dt 1/120, gravity (0,-9.8,0), JGS2_PLAIN,
 * JGS2_JACOBI, omega 1, rel_tol 1e-5, max_sweeps 20000, check_every 8,
 * d_hat 1e-3, kappa 1e4, no planes, no line search, adj_rel_tol 1e-5,
 * adj_max_sweeps 20000, no graph capture. */
void jgs2_default_params(jgs2_params* p);

/* Creates a handle.  Fails with JGS2_E_INVALID on a bad parameter set and
 * JGS2_E_HIP when no gfx950 device is current. */
int32_t jgs2_create(const jgs2_params* p, jgs2_solver** out);
void    jgs2_destroy(jgs2_solver* s);
const char* jgs2_last_error(const jgs2_solver* s);

/* Replaces the parameters; the mesh and material stay.  The correction
 * stays unless dt changes: the rest Hessian it is built from carries the
 * inertia term M / h^2 (Sec. 6 with Sec. 3), so a new dt discards it
 * (JGS2_CUBATURE steps then return JGS2_E_NOT_READY until the next
 * precompute or import).  dt and gravity cannot change inside a step. */
int32_t jgs2_set_params(jgs2_solver* s, const jgs2_params* p);
/* Orders all later work on the HIP stream `stream` (a hipStream_t). */
int32_t jgs2_set_stream(jgs2_solver* s, void* stream);

/* Mesh: nV rest positions X (nV x 3, metres), nT tets (nT x 4) with positive
 * orientation, pinned[nV] (1 = held at its rest position).  Builds vertex
 * adjacency (sub-problems sit at vertices, Sec. 8.1), the greedy colouring
 * of the Gauss-Seidel groups (Sec. 8.1) and the device layout.  Invalidates
 * material, correction and state.  Errors: JGS2_E_INVALID for empty or
 * non-finite input, out-of-range ids, inverted tets or free vertices that
 * belong to no tet. */
int32_t jgs2_upload_mesh(jgs2_solver* s, int32_t nV, const double* X,
                         int32_t nT, const int32_t* tets, const uint8_t* pinned);

/* Bodies: disjoint meshes uploaded as one (concatenated vertex and tet
 * arrays) and solved together in the same launches.  body_of_vertex (nV
 * entries, ids 0..n_bodies-1, in any order) assigns each vertex a body; every
 * body keeps its own residual |g_b| / |g_b(x0)| (FP64, summed in a fixed order
 * over the body's free vertices only) and stops sweeping (its vertices are
 * skipped) once that reaches rel_tol at a residual check, so each body gets
 * exactly the sweeps it would get alone.  upload_mesh resets to one body.
 * The energy line search is refused with more than one body.  Any failure
 * (including a rejected argument) leaves the handle without body tables:
 * steps, residuals and body statistics return JGS2_E_NOT_READY until a
 * later call succeeds. */
int32_t jgs2_set_bodies(jgs2_solver* s, int32_t n_bodies, const int32_t* body_of_vertex);
/* Per body at the last residual check of the current or last step: sweeps
 * done (sweeps, n_bodies entries) and |g_b| / |g_b(x0)| (rel). */
int32_t jgs2_get_body_stats(jgs2_solver* s, int32_t* n_bodies, int32_t* sweeps, double* rel);

/* Launch shape of the plain (and adjoint linear) sweep kernels: lanes_per_vertex
 * in {4, 8, 16, 32} lanes share a vertex's incident tets, block in
 * {64, 128, 256, 512} threads.  Results depend on the shape only through the
 * order of the per-vertex sums.  Default 32 x 256. */
int32_t jgs2_set_tuning(jgs2_solver* s, int32_t lanes_per_vertex, int32_t block);
int32_t jgs2_get_tuning(jgs2_solver* s, int32_t* lanes_per_vertex, int32_t* block);
/* Cache hint for the incidence records the plain and linear sweeps read (one
 * 64-byte record per free vertex and incident tet, read once per sweep):
 * mode 1 streams them with non-temporal loads, which keeps the reused vertex
 * records in L2 when the records outgrow the cache; 0 uses ordinary loads;
 * -1 (default) streams them once they exceed 128 MiB, half of the last-level
 * cache.  Results are bitwise the same in every mode.  Errors: JGS2_E_INVALID
 * for any other mode. */
int32_t jgs2_set_streaming(jgs2_solver* s, int32_t mode);
/* on = 1: a group of check_every coloured Gauss-Seidel sweeps of the plain
 * variant runs as one persistent cooperative launch over every colour and
 * sweep, its blocks (no more than the device keeps resident at once) taking
 * the row blocks of each colour in turn with a grid-wide barrier between
 * colours; 0 (default): one launch per colour (replayed from a captured graph
 * with use_graph).  Results are bitwise the same.  Other variants and
 * orders, the energy line search and profiling use the per-colour launches.
 * Errors: JGS2_E_INVALID for another value; the launch itself reports
 * JGS2_E_HIP if the runtime refuses it. */
int32_t jgs2_set_persistent(jgs2_solver* s, int32_t on);
/* Times `sweeps` sweeps of the first step from the current state in every
 * launch shape (HIP events), keeps the fastest and reports it; the state is
 * left unchanged.  ms (16 entries, may be NULL) receives each shape's time in
 * the order lanes 4, 8, 16, 32 (outer) x block 64, 128, 256, 512 (inner). */
int32_t jgs2_autotune(jgs2_solver* s, int32_t sweeps, int32_t* lanes_per_vertex, int32_t* block, double* ms);

/* Per-tet Young's modulus E [Pa], Poisson ratio nu and density rho
 * [kg/m^3] (stable Neo-Hookean, Sec. 8 / Table 1 caption).  Lumped masses
 * follow.  Invalidates the correction. */
int32_t jgs2_set_material(jgs2_solver* s, const double* E, const double* nu,
                          const double* rho);
/* The same with E_t = exp(log_E[t]): the parametrisation the rollout's
 * stiffness cotangent thetabar refers to.  JGS2_E_INVALID on a non-finite
 * log_E. */
int32_t jgs2_set_material_log_e(jgs2_solver* s, const double* log_E, const double* nu,
                                const double* rho);

/* Precompute of the overshoot correction on the GPU (Secs. 5-6): rest
 * Hessian, its banded Cholesky factor, training poses (smallest
 * eigenvectors), U-bar by Eq. u, greedy NNLS cubature with `samples` samples
 * per vertex drawn from `n_cand` candidates per round (counter-based
 * SplitMix64 keyed by `seed`).  Needed by JGS2_CUBATURE and JGS2_DAMPER.
 * When the handle's variant is JGS2_EXACT it also keeps, for every free
 * vertex, the columns of H-bar^-1 that define its U-bar rows (Eq. u): the
 * lower triangle of 64 x 64-vertex tiles of H-bar^-1 in FP32 over the
 * vertices' bandwidth-reducing order, about nVf^2 x 18 bytes
 * (JGS2_E_OOM when that does not fit), and B_i^-1 per free vertex. */
int32_t jgs2_precompute(jgs2_solver* s, int32_t samples, int32_t n_cand, uint64_t seed);
/* The same with a cache file at `path` (NULL: plain jgs2_precompute).  If the
 * file holds this library build's precompute for the same mesh, pinning,
 * material, dt, variant (exact or not), samples, n_cand and seed (a 64-bit
 * hash of all of them and sizes are checked), the tables are loaded from it
 * and *loaded = 1 (may be NULL); otherwise the precompute runs and the file
 * is written (through a temporary file renamed at the end), *loaded = 0.
 * For the exact variant the file holds every stored H-bar^-1 tile (about
 * nVf^2 x 18 bytes).  A matching file that is cut short is recomputed and
 * rewritten.  JGS2_E_INVALID if the file cannot be written (the tables are
 * still computed). */
int32_t jgs2_precompute_cached(jgs2_solver* s, int32_t samples, int32_t n_cand, uint64_t seed, const char* path,
                               int32_t* loaded);

/* The exact variant's H-bar^-1 tiles after jgs2_precompute: the number of
 * stored tiles (the lower triangle of 64 x 64-vertex tiles), the number a
 * sweep streams under params.exact_drop, the bytes those live tiles hold
 * (rows past the last free vertex excluded), and the bytes of partial sums
 * one sweep writes (1 KB per tile row and per tile column of every 4 x 4
 * super-tile holding a live tile).  Any pointer may be NULL.
 * JGS2_E_NOT_READY without the tiles. */
int32_t jgs2_exact_tiles(jgs2_solver* s, int64_t* n_tiles, int64_t* n_live, double* live_bytes,
                         double* part_bytes);

/* Converts the exact variant's stored H-bar^-1 tiles (Eq. u: U-bar_{i,a} =
 * (H-bar^-1)_{a,i} B_i^-1) to FP16, halving the bytes each sweep streams:
 * every entry is stored divided by its tile's scale (the tile's largest
 * |entry| / 2^15, so that entry maps to 2^15), rounded to nearest; the sweep
 * multiplies in FP32 and sums per position in FP64 as before.  The tiles
 * only form the correction b, whose fixed point (zero gradient) and FP64
 * residual test are unchanged; a step converges to the same tolerance.  The
 * FP32 tiles are freed; a later jgs2_precompute (or a loaded cache) brings
 * FP32 tiles back.  A second call does nothing.  JGS2_E_NOT_READY without
 * tiles, JGS2_E_INVALID inside a step, JGS2_E_OOM if the FP16 copy does not
 * fit beside the FP32 tiles. */
int32_t jgs2_exact_tiles_fp16(jgs2_solver* s);

/* Correction tables in free-vertex order (free vertices ascending by id).
 * For free vertex f with one-ring list ring(f) = its free neighbours in
 * ascending id order (length given by jgs2_get_ring_sizes):
 *   U_ring : for f, k < |ring(f)|: rows Ubar_{f,ring(f)[k]} (3x3 row-major),
 *            packed consecutively over f and k (total sum |ring(f)|).
 *   samples: nVf x S element ids (-1 = unused slot).
 *   weights: nVf x S cubature weights (>= 0).
 *   U_samp : nVf x S x 4 x 3x3: Ubar rows at each sample's 4 corners
 *            (zero rows at pinned corners).
 *   fit    : nVf relative NNLS residuals (export only; may be NULL).
 * import copies these into the device layout (a cache or an external
 * precompute); export reads back what jgs2_precompute produced. */
int32_t jgs2_import_correction(jgs2_solver* s, int32_t S, const double* U_ring,
                               const int32_t* samples, const double* weights,
                               const double* U_samp);
int32_t jgs2_export_correction(jgs2_solver* s, int32_t S, double* U_ring,
                               int32_t* samples, double* weights, double* U_samp,
                               double* fit);
/* Number of free vertices, one-ring sizes per free vertex (nVf entries) and
 * the training-pose eigenvalues of the last precompute (up to 17 entries;
 * *n_poses receives the pose count n_T). */
int32_t jgs2_get_ring_sizes(jgs2_solver* s, int32_t* nVf, int32_t* sizes);
int32_t jgs2_get_poses(jgs2_solver* s, int32_t* n_poses, double* eigenvalues);

/* State: positions x and velocities v (nV x 3) copied from / to the host. */
int32_t jgs2_set_state(jgs2_solver* s, const double* x, const double* v);
int32_t jgs2_get_state(jgs2_solver* s, double* x, double* v);
/* The same for a state that lives in device memory (Sec. 3, Eq. variation:
 * x-hat and its velocity): x and v are device pointers (allocations of the
 * HIP runtime libjgs2 is linked against) to nV x 3 doubles, row-major, read
 * or written on the handle's stream, which the calls wait for; nothing
 * crosses PCIe but a 4-byte flag.  set_state_device returns JGS2_E_INVALID
 * (and leaves no state) if a value is not finite; velocities of pinned
 * vertices are stored as zero.  Results are bitwise those of the host
 * calls. */
int32_t jgs2_set_state_device(jgs2_solver* s, const double* x, const double* v);
int32_t jgs2_get_state_device(jgs2_solver* s, double* x, double* v);

/* One implicit-Euler step (Sec. 3): z = xhat + h vhat + h^2 g, x0 = xhat,
 * sweeps until |g|/|g(x0)| <= rel_tol or max_sweeps, then v = (x - xhat)/h.
 * Returns JGS2_NOT_CONVERGED (state and velocity kept, stats filled) when
 * some body is still above rel_tol after max_sweeps.  On JGS2_E_DIVERGED /
 * NONFINITE / INFEASIBLE the state is left at the start of the step. */
int32_t jgs2_step(jgs2_solver* s, jgs2_step_stats* stats);
/* The same step in pieces: begin (z, x0, r0), n sweeps (relative residual
 * of the resulting iterate in *rel_res, may be NULL), end (velocity). */
int32_t jgs2_begin_step(jgs2_solver* s);
int32_t jgs2_iterate(jgs2_solver* s, int32_t n_sweeps, double* rel_res);
int32_t jgs2_end_step(jgs2_solver* s);

/* |g| over free DOFs at the current iterate, and |g| / r0, with g the
 * gradient of the incremental potential E of Eq. variation (inertia of
 * Sec. 3, elasticity, plane barriers of Eq. barrier), evaluated in FP64.
 * The paper's own measure, the last sweep's |dx| (Sec. 8, Table 1), is in
 * jgs2_step_stats.dx_norm.  JGS2_E_NOT_READY without mesh, material,
 * state or (non-plain variants) correction. */
int32_t jgs2_residual(jgs2_solver* s, double* abs_res, double* rel_res);
/* Differentiable rollout.  The paper defines the forward step only; its
 * derivative is taken through the step's optimality condition
 * G(x_{n+1}; x_n, v_n, theta) = grad E = 0 (Sec. 3, Eq. variation) with
 * theta_e = log E_e per tet.  For cotangents (xbar_{n+1}, vbar_{n+1}) of a
 * step's outputs, with H the Hessian of E at x_{n+1}:
 *     H y = xbar_{n+1} + vbar_{n+1} / h
 *     thetabar_e -= y_e . grad_{x_e}(V_e Psi_e(x_{n+1}))
 *     xbar_n = M y / h^2 - vbar_{n+1} / h,   vbar_n = M y / h
 * (rows of pinned vertices are zero).  H y = b is solved by linear
 * per-vertex sweeps in the configured order and omega: the residual
 * r = H y - b replaces the gradient and each vertex takes the 3x3 step
 * -A_i^-1 r_i with A_i = H_ii, as in the forward plain sweeps.
 *
 * jgs2_rollout runs n_steps forward steps from the current state (as
 * jgs2_step, same parameters) and keeps the state at every ckpt_every-th
 * step on the device; it returns JGS2_NOT_CONVERGED (rollout kept) when a
 * step stopped at max_sweeps.  jgs2_rollout_backward pulls (xbar_N, vbar_N)
 * (nV x 3; vbar may be NULL for zero) back through the whole rollout,
 * recomputing the steps of each checkpoint segment from its checkpoint, and
 * writes thetabar (nT, the cotangent of theta_e = log E_e), xbar_0 and
 * vbar_0 (nV x 3 each) and ubar (3: the cotangent of one initial velocity
 * shared by all free vertices, i.e. vbar_0 summed over free vertices in
 * ascending order, FP64); any output may be NULL.  The state is left at the
 * end of the rollout.  set_state, set_material, set_params and upload_mesh
 * discard the rollout (JGS2_E_NOT_READY).  A recomputed step or adjoint
 * solve that diverges (residual past 1e8 x its scale) or turns non-finite
 * returns JGS2_E_DIVERGED / JGS2_E_NONFINITE; one that stops at its sweep
 * cap above its tolerance makes the call return JGS2_NOT_CONVERGED with
 * every output written, and stats->max_rel_res reports the largest final
 * relative residual of the adjoint solves. */
int32_t jgs2_rollout(jgs2_solver* s, int32_t n_steps, int32_t ckpt_every, jgs2_step_stats* last);
int32_t jgs2_rollout_backward(jgs2_solver* s, const double* xbar, const double* vbar, double* thetabar,
                              double* xbar0, double* vbar0, double* ubar, jgs2_adjoint_stats* stats);

/* Incremental potential E of Eq. variation at the current iterate: the
 * inertia term (1/2h^2)|M^(1/2)(x - z)|^2 of Sec. 3, the stable Neo-Hookean
 * energy and the log barriers of Eq. barrier (infinite for a vertex on or
 * behind a plane); an FP64 sum of FP32 element terms.  JGS2_E_NOT_READY as
 * for jgs2_residual. */
int32_t jgs2_energy(jgs2_solver* s, double* e);
/* Allocation-free variant of jgs2_energy, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, hosts
 * that forbid hipMalloc.  Same result as jgs2_energy (the same kernels and
 * summation order).  The per-block partial sums and the total live in a
 * file-scope device array of JGS2_NOALLOC_MAX_PARTIALS + 1 doubles (512 KiB)
 * that every GPU the library runs on holds until the process ends; its
 * address on a device is taken by the first jgs2_create on that device.
 * Meshes with more than 256 * JGS2_NOALLOC_MAX_PARTIALS tets or free vertices
 * are refused with JGS2_E_INVALID.  All calls on one GPU share the array, so
 * calls that overlap on one GPU (several threads or streams) race.  Calls no
 * hipMalloc or hipFree; copies the total to *e (host) and waits for the
 * handle's stream; no profiling events are recorded for its launches. */
#define JGS2_NOALLOC_MAX_PARTIALS 65536
int32_t jgs2_energy_noalloc(jgs2_solver* s, double* e);
/* Assembled gradient g (nV x 3, zero at pinned vertices) and per-vertex
 * rotations R (nV x 3x3 row-major, identity at pinned vertices) at the
 * current iterate: the outputs of the first sweep phase. */
int32_t jgs2_get_phase1(jgs2_solver* s, double* g, double* R);
/* Greedy colour per vertex (-1 for pinned) and the colour count: the
 * independent groups of the Gauss-Seidel order of Sec. 8.1 (each colour is
 * the smallest one unused by the vertex's lower-id free neighbours), the
 * order of the GS sweeps.  color has nV entries (may be NULL). */
int32_t jgs2_get_coloring(jgs2_solver* s, int32_t* color, int32_t* n_colors);

/* Per-kernel device timing with HIP events on the handle's stream.  While
 * profiling is on, every launch of a library kernel is bracketed by an event
 * pair; jgs2_kernel_times() returns, per kernel id below, the accumulated
 * milliseconds and launch counts since profiling was (re)enabled.  ms and
 * launches point to JGS2_NKERNELS entries each.  Profiling adds a small gap
 * between launches, not to the kernels themselves. */
#define JGS2_K_PHASE1    0   /* gradient, rotations, |g|^2 partials */
#define JGS2_K_PHASE2    1   /* cubature-corrected local solves */
#define JGS2_K_PLAIN     2   /* plain per-vertex Newton, fused */
#define JGS2_K_COMMIT    3
#define JGS2_K_REDUCE    4
#define JGS2_K_PREDICT   5
#define JGS2_K_VELOCITY  6
#define JGS2_K_ENERGY    7
#define JGS2_K_LINEAR    8   /* adjoint: linear per-vertex sweep on H y = b */
#define JGS2_K_PARAMGRAD 9   /* adjoint: per-tet stiffness gradient */
#define JGS2_K_ADJVEC    10  /* adjoint: mass products, next right-hand side */
#define JGS2_K_DAMPER    11  /* damper-corrected local solves, fused with the gather */
#define JGS2_K_ROT       12  /* per-vertex rotations alone (the damper sweeps' start) */
#define JGS2_K_EXACT     13  /* exact-subspace local solves (Hessian term, 3x3 solve) */
#define JGS2_K_HVEC      14  /* rest-frame gradients R_a^T g_a in the tiles' position order */
#define JGS2_K_SYMV      15  /* H-bar^-1 tiles against those gradients, both ways per tile */
#define JGS2_K_YSUM      16  /* tile partials summed per position */
#define JGS2_NKERNELS    17
int32_t jgs2_set_profiling(jgs2_solver* s, int32_t on);
int32_t jgs2_kernel_times(jgs2_solver* s, double* ms, int64_t* launches);

/* Debugging aid, not part of the method.  The library built with
 * JGS2_BOUNDS_CHECK (libjgs2_bounds.so, `python -m paper_2506_06494_amd.build
 * --bounds`) checks, inside the sweep kernels (gradient gather, exact-variant
 * tile product, sums and local solves, plain, linear and damper sweeps), every
 * index read from a table before it is used: list entries, vertex, tet and
 * position ids, one-ring slots, super-tile ids and partial ranges.  A failed
 * check keeps the access inside its buffer (index 0 is used instead) and
 * records the first failure: the kernel source line, the index and its
 * extent; jgs2_step then fails with JGS2_E_BOUNDS and names them.
 * jgs2_bounds_report copies that record (line 0: no failure; any pointer may
 * be NULL) and clears it when clear != 0.  jgs2_bounds_selftest records a
 * failure (index 1 of extent 0) from a kernel that touches no buffer, to test
 * the reporting path.  In other builds both return JGS2_E_INVALID. */
int32_t jgs2_bounds_report(jgs2_solver* s, int32_t* line, int64_t* index, int64_t* extent, int32_t clear);
int32_t jgs2_bounds_selftest(jgs2_solver* s);

#ifdef __cplusplus
}
#endif
#endif /* JGS2_H */
