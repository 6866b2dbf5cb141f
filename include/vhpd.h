/*
 * vhpd -- projective dynamics for volumetric homogenization on MI355X (gfx950).
 *
 * C ABI of the native library libvhpd.so.  One simulated garment is a
 * tetrahedral mesh with a per-element material (gamma_s, gamma_v), simulated
 * by the projective-dynamics (PD) step of the paper "Volumetric Homogenization
 * for Knitwear Simulation", Sec. 7:
 *
 *   - time discretisation (Sec. 7): the implicit-Euler target
 *       y = x* + dt v* + dt^2 g,
 *   - local step (Sec. 7.1, Eq. pd_local, Eq. vol_pre): per element the polar
 *     rotation R(F_e) and the nearest volume-preserving V(F_e),
 *   - global step (Sec. 7.1): the constant SPD system K x = b,
 *       K = M/dt^2 + sum_e V_e (gs_e + gv_e) B_e^T (D^T:D) B_e,
 *       b = M y/dt^2 + sum_e V_e B_e^T D^T:(gs_e R_e + gv_e V_e),
 *     solved by domain decomposition (Sec. 7.2): per-subdomain interior
 *     Cholesky solves plus the interface (Schur complement) solve that the
 *     boundary modes Psi_d = -(K_d^ii)^{-1} K_d^ib of Eq. (cms_boundary) and the
 *     shared boundary unknowns of Eq. (global_subspace) lead to.
 *   - BDF1 velocity v = (x_{n+1} - x_n)/dt after pd_iters local/global
 *     iterations started from x^(0) = y.
 *
 * Conventions for every entry point:
 *   - Return value: VH_OK (0) on success, a negative VH_E* code on failure; the
 *     message of the last failure on the calling thread is vh_last_error().
 *     No C++ exception crosses this boundary.
 *   - Host arrays passed in are read during the call and copied; the caller
 *     keeps ownership.  Host arrays passed out are written during the call.
 *   - Layouts are C-contiguous row-major: positions [nv][3] float64,
 *     tets [nt][4] int32 (vertex ids, positively oriented), per-element
 *     arrays [nt], per-vertex arrays [nv].
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     Device work is enqueued on it; entry points that return host data
 *     synchronise it.
 *   - Handles are opaque and owned by the library; destroy them with the
 *     matching *_destroy call.  A handle is not thread-safe: calls on one
 *     handle must not overlap.
 */
#ifndef VHPD_H
#define VHPD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    VH_OK = 0,
    VH_EINVAL = -1,   /* invalid argument (sizes, ids, orientation, gamma < 0, ...) */
    VH_ENOMEM = -2,   /* host or device allocation failed, or over the HBM budget */
    VH_ENOTSPD = -3,  /* a non-positive pivot in the FP64 factorization */
    VH_ESTATE = -4,   /* call out of order (e.g. step before prefactor) */
    VH_ENUMERIC = -5, /* a NaN/Inf appeared in the device state */
    VH_EDEVICE = -6   /* a HIP runtime call failed */
};

typedef struct vh_ctx vh_ctx;
typedef struct vh_mesh vh_mesh;

/* Message of the last failed call on this thread ("" if none). */
const char* vh_last_error(void);

/* Context: one GPU.  hbm_budget_bytes bounds the device memory the library
 * holds for all meshes of this context (0 = unlimited).  The device is made
 * current on the calling thread. */
int vh_ctx_create(vh_ctx** out, int device, size_t hbm_budget_bytes);
/* Destroys the context and every mesh still alive on it (their handles become
 * invalid). */
int vh_ctx_destroy(vh_ctx* ctx);
/* Device bytes currently held by the context's meshes. */
int vh_ctx_hbm_in_use(const vh_ctx* ctx, size_t* bytes);
/* Change the budget (0 = unlimited).  Memory already held is kept; later
 * allocations and admissions are checked against the new value. */
int vh_ctx_set_hbm_budget(vh_ctx* ctx, size_t hbm_budget_bytes);

/* Execution settings of a context (no process-wide switches exist).
 *   use_graphs:        1 (default): a mesh replays its frame as a captured HIP
 *                      graph, and a server launches captured frame graphs;
 *                      0: every launch of a frame is enqueued directly
 *                      (the same kernels and arguments, hence the same results);
 *   iface_lanes32_min, iface_lanes64_min (defaults 96, 384, both >= 1):
 *                      an interface-solve phase whose mean task length (rows
 *                      of the factor block a task sweeps) reaches these values
 *                      runs 32 / 64 lanes per task, else 16.  Results do not
 *                      depend on the lane count beyond FP64 summation order;
 *   thin_separators:   1 (default): a separator vertex whose neighbours lie
 *                      under one side of its separator only is eliminated on
 *                      that side (a smaller interface); 0: every vertex shared
 *                      by elements of two subdomains is an interface vertex;
 *   iface_merge_max_cols (default 3000, >= 0): a separator at odd depth of the
 *                      bisection tree joins its parent's block when the merged
 *                      block has at most this many columns (fewer interface
 *                      launches, more stored values); 0: no merging.
 * These four change the plan, hence rounding, not the solution.
 *   cms_modes (default 0, >= 0): 0 solves the global step exactly (interior
 *                      Cholesky solves, Sec. 7.2 with the interior modes made
 *                      exact).  > 0 selects the paper's inexact component mode
 *                      synthesis: per subdomain the cms_modes eigenvectors of
 *                      the interior block with the smallest eigenvalues next
 *                      to the exact boundary modes of Eq. cms_boundary, the
 *                      reduced solve of Eq. global_subspace applied to each PD
 *                      iteration's residual, then
 *   cms_sweeps (default 10, >= 0) Jacobi sweeps of the global system with
 *                      Chebyshev weights.  The CMS solve is approximate: it
 *                      changes the trajectory (an error to report against the
 *                      exact solve); it needs refine_steps == 0 and is not
 *                      differentiated by the adjoint entry points.
 *   interior_desc_table (default 64, 1..64): the interior solves copy the
 *                      descriptors of a subdomain's first this many program
 *                      chunks to LDS at kernel start and read later ones from
 *                      global memory (a subdomain's program rarely exceeds 40
 *                      chunks; a smaller table exercises the global reads).
 *                      Results do not depend on it.
 * vh_ctx_set_config validates and copies *cfg (VH_EINVAL on out-of-range
 * values); it applies to meshes prefactored and servers opened afterwards, and
 * use_graphs also to later vh_mesh_step calls of meshes already resident. */
typedef struct vh_config {
    int32_t use_graphs;
    int32_t iface_lanes32_min, iface_lanes64_min;
    int32_t thin_separators;
    int32_t iface_merge_max_cols;
    int32_t cms_modes, cms_sweeps;
    int32_t interior_desc_table;
} vh_config;
int vh_ctx_get_config(const vh_ctx* ctx, vh_config* cfg);
int vh_ctx_set_config(vh_ctx* ctx, const vh_config* cfg);

/* Mesh: rest positions X [nv][3] (metres) and tets [nt][4].  Every tet must
 * have positive rest volume det([X1-X0, X2-X0, X3-X0])/6 > 0 (VH_EINVAL
 * otherwise; tets are never reoriented silently).  Sec. 5 defines the per-tet
 * operator D and volume V_e this uses. */
int vh_mesh_create(vh_ctx* ctx, vh_mesh** out, const double* rest_xyz, int32_t nv,
                   const int32_t* tets, int32_t nt);
int vh_mesh_destroy(vh_mesh* mesh);

/* Material and step settings.  gamma_s, gamma_v [nt] >= 0 (Pa; Eq. energy,
 * Sec. 6.3 requires gamma >= 0); mass [nv] lumped nodal masses, > 0 on every
 * free vertex (kg); pinned [nv] 1 = Dirichlet at the rest position; gravity
 * [3] (m/s^2); dt > 0 (s); pd_iters >= 1 local/global iterations per step.
 * Invalidates any previous factorization and resets the state to rest with
 * zero velocity. */
int vh_mesh_set_params(vh_mesh* mesh, const double* gamma_s, const double* gamma_v,
                       const double* mass, const uint8_t* pinned, const double* gravity,
                       double dt, int32_t pd_iters);

/* Arithmetic of the step (precision_mode of vh_mesh_prefactor).  The one
 * mode: local step and interior subdomain solves in FP32 with FP32
 * accumulation; factorizations, interface (Schur complement) solve, residual
 * and refinement in FP64; state x, v in FP64. */
enum { VH_PRECISION_MIXED = 0 };

/* Prefactor (host FP64): partitions the elements into n_subdomains (a power of
 * two, >= 1) by recursive breadth-first bisection, orders each subdomain's
 * interior by nested dissection and the interface by the bisection tree,
 * factors the global matrix (interior Cholesky factors and the interface
 * Schur complement), and uploads it.  refine_steps (>= 0) extra solves of the
 * global system against its FP64 residual are done every PD iteration.
 * precision_mode must be VH_PRECISION_MIXED (VH_EINVAL otherwise).
 * VH_ENOTSPD on a non-positive pivot, VH_ENOMEM over the HBM budget. */
int vh_mesh_prefactor(vh_mesh* mesh, int32_t n_subdomains, int32_t refine_steps,
                      int32_t precision_mode);

/* New per-element stiffness gamma_s, gamma_v [nt] (>= 0, as in
 * vh_mesh_set_params) for a prefactored mesh, as a fitting loop changes it
 * (Sec. 6).  The global matrix of Sec. 7.1 depends on gamma only through its
 * values: the partition, orderings, supernodes and solve programs are kept,
 * the element weights, the matrix values and the numeric FP64 factorization
 * are redone on the host, and the device factor is overwritten in place, so
 * captured frame graphs stay valid.  The state x, v is kept; adjoint
 * checkpoints are dropped.  VH_ESTATE unless prefactored (or while the server
 * drives the mesh); VH_EINVAL with the CMS solve selected (vh_mesh_prefactor
 * rebuilds its modes); VH_ENOTSPD on a non-positive pivot, after which the
 * mesh needs vh_mesh_prefactor. */
int vh_mesh_refactor(vh_mesh* mesh, const double* gamma_s, const double* gamma_v);

/* Advance n_frames time steps on `stream` (asynchronous). */
int vh_mesh_step(vh_mesh* mesh, int32_t n_frames, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * n_frames steps as vh_mesh_step, with the same kernels and the same results,
 * but the work buffers of those kernels (force partials, residual, interior
 * and interface work vectors, contribution slots, the launch record) taken
 * from one fixed device array of VH_NOALLOC_SCRATCH_BYTES per GPU, which the
 * library holds from its load until the process ends; the call allocates
 * nothing (no hipMalloc, no graph instantiation: every launch is enqueued on
 * `stream` directly).  The mesh (prefactored, not in a server) keeps its state
 * and factors in its own memory.  VH_EINVAL when the mesh's work buffers need
 * more than the array holds (about 14 MB for the 390,400-tet shell).  Every
 * call on one GPU uses that GPU's one array: calls that overlap on a device
 * (other streams or threads) race and must be serialised by the caller.  The
 * array is cleared at the start of each call. */
#define VH_NOALLOC_SCRATCH_BYTES ((size_t)16 << 20)
int vh_mesh_step_noalloc(vh_mesh* mesh, int32_t n_frames, void* stream);

/* Copy the state to host x, v [nv][3] (float64); synchronises `stream` and
 * returns VH_ENUMERIC if the state holds a NaN/Inf. */
int vh_mesh_read_state(vh_mesh* mesh, double* x, double* v, void* stream);
/* Overwrite the state from host x, v [nv][3]; pinned vertices keep their rest
 * position and zero velocity whatever is passed. */
int vh_mesh_write_state(vh_mesh* mesh, const double* x, const double* v, void* stream);
/* Same with device pointers (e.g. torch tensors' data_ptr), [nv][3] float64 in
 * user vertex order; asynchronous on `stream`. */
int vh_mesh_read_state_device(vh_mesh* mesh, double* x_dev, double* v_dev, void* stream);
int vh_mesh_write_state_device(vh_mesh* mesh, const double* x_dev, const double* v_dev,
                               void* stream);

typedef struct vh_mesh_info {
    int32_t nv, nt, n_free, n_interior, n_interface, n_subdomains;
    int32_t n_supernodes, n_coarse_levels, max_interior_phases;
    int64_t nnz_interior;   /* stored entries of the FP32 interior factor blocks */
    int64_t nnz_coarse;     /* stored entries of the FP64 interface factor blocks */
    size_t device_bytes;
    double prefactor_seconds;
    int64_t n_partials;     /* per-(local-step workgroup, vertex) force partials */
    /* algorithmic bytes moved by one launch of each kernel class (the
     * interface: one whole solve, all its launches): data each kernel must
     * read or write once, without re-reads */
    int64_t bytes_local, bytes_residual, bytes_interior_fwd, bytes_interface, bytes_interior_bwd;
    int32_t interface_launches;   /* kernel launches per interface solve */
} vh_mesh_info;
int vh_mesh_get_info(const vh_mesh* mesh, vh_mesh_info* info);

/* Projection regimes met by the local step (Sec. 7.1, Eq. vol_pre), counted
 * per element evaluation (one element in one PD iteration; the adjoint's
 * re-evaluations count too) since the last reset (prefactor resets them):
 *   clamped       a projected singular value fell below 0.01: it was set to
 *                 0.01, frozen, and the other axes solved again for the
 *                 remaining product;
 *   inverted      sigma_3 <= 0 (det F <= 0);
 *   det_ge2       every sigma_i > 0 and det F >= 2, where stationary points
 *                 with one axis on the minus root of the Lagrange condition
 *                 exist and are searched;
 *   squash        such a point was the nearest one (also in a clamp re-solve);
 *   no_plus_root  the branch with every axis on its plus root had no root.
 * Synchronises `stream`; reset != 0 zeroes the counters after reading. */
typedef struct vh_regime_counts {
    uint64_t clamped, inverted, det_ge2, squash, no_plus_root;
} vh_regime_counts;
int vh_mesh_regime_counts(vh_mesh* mesh, vh_regime_counts* out, int32_t reset, void* stream);

/* Per-kernel timing with HIP events recorded on the step's stream around each
 * launch group of a kernel class (bit c of class_mask enables class c):
 *   0 predictor, 1 local step, 2 (unused: the PD iterations form the residual
 *   inside the interior forward solve), 3 interior forward solve (with the
 *   residual gather of the PD iteration, when it forms it), 4 interface solve
 *   (all tree levels), 5 interior backward solve + update, 6 refinement
 *   residual, 7 velocity.
 * vh_mesh_profile resets the record and sets the mask (0 = off);
 * vh_mesh_profile_read synchronises and returns, per class, the summed
 * milliseconds ms[8] and the number of timed groups launches[8] since then. */
#define VH_PROFILE_CLASSES 8
int vh_mesh_profile(vh_mesh* mesh, uint32_t class_mask);
int vh_mesh_profile_read(vh_mesh* mesh, double* ms, int64_t* launches);

/* Launch one kernel class (1 local step, 2 residual gather as a launch of
 * its own, 3 interior forward with the residual gather as the PD iterations
 * run it, 4 all interface phases of one solve, 5 interior backward without
 * update, 6 interior forward reading the residual) `reps` times back to back
 * on `stream`, on the mesh's current data, for timing with events around the
 * call.  The local step and residual overwrite only their outputs; the solve
 * kernels only their work vectors and the residual. */
int vh_mesh_time_kernel(vh_mesh* mesh, int32_t kernel_class, int32_t reps, void* stream);

/* ---- Embedded points (Eq. m2y): positions of points carried by the mesh,
 * e.g. the vertices of yarn curves, phi(x) = N x, where row i of N holds the
 * linear shape functions N_0..N_3 of point i's tet evaluated at the point's
 * rest position (natural coordinates N_1..3 = Dm^{-1} (X^i - X_0), N_0 =
 * 1 - N_1 - N_2 - N_3, Dm the tet's rest edge matrix).  Points outside their
 * tet are extrapolated linearly. ---- */

/* Set (replace) the embedded points: tet[n_points] user element indices and
 * rest_xyz[n_points][3] rest positions (float64), both copied.  n_points = 0
 * clears.  N is formed in FP64 on the host and stored as FP32 next to the
 * tet's four vertex ids (32 bytes per point on the device, plus a 24-byte
 * output row; charged to the HBM budget when the mesh is resident).
 * VH_EINVAL on n_points < 0, null arrays, a tet index out of range or a
 * non-finite rest coordinate. */
int vh_mesh_set_embedding(vh_mesh* mesh, int32_t n_points, const int32_t* tet, const double* rest_xyz);
/* Positions of the embedded points for the current state, [n_points][3]
 * float64 in the order given: into host `out` (synchronises `stream`), or into
 * device `out_dev` (asynchronous on `stream`).  The mesh must be prefactored
 * and, when it is driven by the server, have no frames pending (VH_ESTATE). */
int vh_mesh_embed(vh_mesh* mesh, double* out, void* stream);
int vh_mesh_embed_device(vh_mesh* mesh, double* out_dev, void* stream);

/* ---- Discrete adjoint with respect to gamma_s (gradients of a trajectory).
 *
 * The forward map is n_frames PD steps (Sec. 7) from (x0, v0); the adjoint
 * reverses every local/global iteration: with lambda = K^{-1} xbar^(k+1),
 * gamma_s gets V_e <G_e lambda, R_e(x^(k)) - F_e(x^(k+1))> (the right-hand side
 * and K both depend on gamma_s, Sec. 7.1) and xbar^(k) = sum_e G_e^T
 * J_P(F_e(x^(k))) [G_e lambda], the derivative of the projections of Eq.
 * pd_local and Eq. vol_pre (FP32, like the local step); then the predictor and
 * the BDF1 velocity are reversed.  A singular value frozen by the clamp has
 * zero derivative and the others follow their re-solved product; the
 * projections are counted like in the forward step. ---- */

/* Run n_frames (>= 1) steps from the host state x0, v0 [nv][3] (user order)
 * on `stream`, keeping (x, v) on the device every ckpt_every (>= 1) frames
 * (2 * ceil(n_frames / ckpt_every) * nv * 3 doubles, charged to the budget
 * until the next call, set_params or destroy); x_final [nv][3] receives the
 * final positions (the stream is synchronised). */
int vh_mesh_adjoint_forward(vh_mesh* mesh, const double* x0, const double* v0, int32_t n_frames,
                            int32_t ckpt_every, double* x_final, void* stream);
/* Given dLoss/dx_final (xbar [nv][3]) and optionally dLoss/dv_final (vbar,
 * NULL = 0), write dLoss/dgamma_s [nt] (user element order) for the last
 * vh_mesh_adjoint_forward.  Each checkpoint segment is replayed once, keeping
 * its iterates (ckpt_every * (pd_iters + 1) * nv * 3 doubles of scratch); the
 * mesh state is left at an unspecified frame.  Pinned rows of xbar, vbar are
 * ignored.  VH_ESTATE without a preceding forward. */
int vh_mesh_adjoint_backward(vh_mesh* mesh, const double* xbar, const double* vbar, double* grad_gamma_s,
                             void* stream);

/* ---- Adjoint Gauss-Newton direction for gamma_s (Sec. 6.2, Eq. gn, Eq. agn).
 *
 * At an equilibrium x_eq of one implicit Euler step of the mesh (the point the
 * PD iteration of Sec. 7.1 converges to: g(x, gamma) = M (x - y)/dt^2 +
 * sum_e G_e^T (w_s (F - R) + w_v (F - V)) = 0, Eq. g), for the loss
 * eps = 1/2 ||x - x_target||^2 over the free vertices:
 *   grad = d eps / d gamma_s = -B^T lambda,  A lambda = x_eq - x_target
 *       (Eq. adjoint_state, Eq. adjoint_state_solve; A = dg/dx, B = dg/dgamma_s),
 *   direction d:  (B^T A^{-1} A^{-1} B + kappa I) d = -grad
 *       (Eq. gn with the Levenberg-Marquardt kappa I; the same d solves the
 *       saddle system of Eq. agn with kappa I in its gamma block).
 * d is found by conjugate gradients in gamma space (at most max_outer
 * iterations, until the residual is outer_tol times the first one); every
 * product takes two solves with A by conjugate gradients preconditioned with
 * the step's decomposed solve (FP64 vectors; the projection Jacobian and the
 * interior solves in FP32 as in the step).  x_eq, x_target [nv][3] (user
 * order; pinned rows ignored); grad_gamma_s, direction [nt] (user element
 * order); stats (may be NULL).  kappa >= 0 (absolute; the GN matrix scales
 * like (dx/dgamma)^2), 0 < outer_tol < 1, max_outer >= 0.  The mesh's state is
 * not changed.  VH_ENUMERIC if A or the damped GN matrix is not positive
 * definite along a search direction (e.g. at a strongly compressed state). */
typedef struct vh_gn_stats {
    int32_t outer_iters;           /* conjugate-gradient iterations in gamma space */
    int64_t inner_iters;           /* preconditioned CG iterations of all solves with A */
    double outer_rel_residual;     /* final |r| / |r_0| of the gamma-space iteration */
    double inner_rel_residual_max; /* worst final relative residual of a solve with A */
} vh_gn_stats;
int vh_mesh_gn_direction(vh_mesh* mesh, const double* x_eq, const double* x_target, double kappa,
                         int32_t max_outer, double outer_tol, double* grad_gamma_s, double* direction,
                         vh_gn_stats* stats, void* stream);

/* ---- Entry points that run one part of the step, for testing each kernel
 * against a reference.  All arrays are host arrays in user vertex order. ---- */

/* Local step (Sec. 7.1) at positions x [nv][3]: per tet e, writes the
 * residual stress T_e = gs_e V_e (R_e - F_e) + gv_e V_e (V_e - F_e) [nt][9]
 * (row-major 3x3, float64 copy of the FP32 result) and, if not NULL, the signed
 * singular values sigma [nt][3] and projected ones s [nt][3]. */
int vh_debug_local_step(vh_mesh* mesh, const double* x, double* T, double* sigma, double* s);

/* Residual of the global system (Sec. 7.1) at positions x with inertial
 * target y: r = b(x) - K x on free vertices, written to r [nv][3] (pinned rows
 * are 0).  Uses the local-step and scatter kernels. */
int vh_debug_residual(vh_mesh* mesh, const double* x, const double* y, double* r);

/* The same residual as the PD iterations form it: the local step, then the
 * interior forward solve, whose first stage gathers r (each subdomain's
 * workgroup its interior rows and an equal share of the interface rows)
 * before it solves.  Writes r [nv][3] (pinned rows 0); equal bit for bit to
 * vh_debug_residual's. */
int vh_debug_residual_in_solve(vh_mesh* mesh, const double* x, const double* y, double* r);

/* The scatter of the local step's corner forces by element colouring, a
 * cross-check of the atomic-free partial sums the step uses (Sec. 7.1's
 * assembly of the global right-hand side): the tets are coloured greedily so
 * that no two of a colour share a free vertex, and one launch per colour adds
 * each tet's four corner forces (formed from the local step at x [nv][3])
 * straight into FP32 vertex sums.  Writes the elastic forces f [nv][3]
 * (pinned rows 0) -- vh_debug_residual with y = x gives the same forces up to
 * FP32 summation order -- and, if not NULL, the colour count.  VH_EINVAL when
 * more than 64 colours would be needed. */
int vh_debug_scatter_colored(vh_mesh* mesh, const double* x, double* f, int32_t* n_colors);

/* The resident interface factor values (the FP64 blocks of the interface
 * supernodes the interface phases read: rows of [Ti; W_B] and columns of
 * [Ti; -W_B], or a root's A = Ti^T Ti), copied from the device.  With out ==
 * NULL, *count receives their number; otherwise *count must equal it. */
int vh_debug_interface_factor(vh_mesh* mesh, double* out, int64_t* count);

/* Solve K_ff d = rhs with the decomposed solver; rhs and d are [nv][3]
 * (pinned rows ignored on input, 0 on output). */
int vh_debug_solve(vh_mesh* mesh, const double* rhs, double* d);

/* ---- Serving: continuous batching of step requests across meshes ----
 *
 * Not part of the paper's method: a request loop around the step above.  A
 * context has at most one server.  Meshes handed to it are prefactored on the
 * host at once and wait, in the order they were added, until their device
 * memory fits in the context's HBM budget; then they are uploaded
 * ("resident").  Step requests (n frames of one mesh) are queued per mesh and
 * run in order.  The caller drives the server from one thread with
 * vh_serve_tick / vh_serve_drain; launches go to the server's own stream.
 *
 * Times are seconds on the server clock, which starts at vh_serve_open.  A
 * request's latency runs from its arrival to the completion, on the GPU, of
 * its last frame (the GPU clock is aligned to the host clock at open). */

enum {
    /* each launch steps one frame of every resident mesh with a request
     * waiting: one captured frame graph over all resident meshes, with the
     * meshes that have no request masked off in its kernels (a launch of a
     * single mesh uses that mesh's own frame graph) */
    VH_SERVE_BATCHED = 0,
    /* each launch steps one frame of one mesh with its own frame graph (plain
     * stepping, one mesh at a time; the baseline for batching) */
    VH_SERVE_SEQUENTIAL = 1
};

/* Open the server.  max_in_flight (1..64) bounds the launches enqueued ahead
 * of the GPU; max_batch (>= 0, 0 = no limit) bounds the meshes per batched
 * launch. */
int vh_serve_open(vh_ctx* ctx, int32_t mode, int32_t max_in_flight, int32_t max_batch);
/* Wait for every launch and close the server.  Meshes still in it leave it
 * as they are (resident meshes stay on the device and can be stepped with
 * vh_mesh_step again). */
int vh_serve_close(vh_ctx* ctx);
/* Hand a mesh (parameters set) to the server.  A mesh already on the device
 * (prefactored, not released) is resident at once.  Otherwise it is queued
 * for admission, after being factored on the host now (as vh_mesh_prefactor
 * with n_subdomains, refine_steps) unless it kept its host factorization
 * from an earlier prefactor or server (n_subdomains and refine_steps are then
 * ignored, and its state restarts at rest when admitted); VH_ENOMEM if it
 * alone exceeds the budget.  All meshes of a server need equal pd_iters and
 * refine_steps (VH_EINVAL otherwise).  While a mesh is in the server,
 * vh_mesh_step, the debug, timing and profiling calls on it return
 * VH_ESTATE, and its state may be read or written only while it has no
 * frames outstanding. */
int vh_serve_add(vh_ctx* ctx, vh_mesh* mesh, int32_t n_subdomains, int32_t refine_steps);
/* Queue a request for n_frames (>= 1) frames of mesh; t_arrival is its
 * arrival time on the server clock (< 0: now).  *ticket identifies it. */
int vh_serve_submit(vh_ctx* ctx, vh_mesh* mesh, int32_t n_frames, double t_arrival, uint64_t* ticket);
/* One scheduling round: retire completed launches, free released meshes,
 * admit waiting meshes that fit, then enqueue launches while fewer than
 * max_in_flight are outstanding.  With wait != 0 and nothing enqueued, block
 * until the oldest outstanding launch completes.  *n_launched (may be NULL)
 * receives the launches enqueued. */
int vh_serve_tick(vh_ctx* ctx, int32_t wait, int32_t* n_launched);
/* Tick until every request has completed.  VH_ESTATE if requests wait for
 * meshes that cannot be admitted next to the resident ones. */
int vh_serve_drain(vh_ctx* ctx);
/* The mesh takes no more requests; once its queued frames have completed its
 * device memory is freed (making room for waiting meshes), it leaves the
 * server, and its last state stays readable with vh_mesh_read_state.  A mesh
 * still waiting for admission with requests is admitted and runs them
 * first. */
int vh_serve_release(vh_ctx* ctx, vh_mesh* mesh);
/* *done = 1 once every frame of the request has completed, with *latency_s
 * (may be NULL) its latency; otherwise *done = 0 and *latency_s = -1. */
int vh_serve_poll(vh_ctx* ctx, uint64_t ticket, int32_t* done, double* latency_s);
/* Current time on the server clock. */
int vh_serve_now(vh_ctx* ctx, double* t);

/* Launch the batched local step (kernel_class 1) or residual gather (2)
 * over every resident mesh `reps` times back to back on `stream`, after the
 * server's own launches have completed, for timing with events around the
 * call (batched servers only).  Each launch overwrites only that kernel's
 * outputs. */
int vh_serve_time_kernel(vh_ctx* ctx, int32_t kernel_class, int32_t reps, void* stream);

/* Restart the statistics window: completed requests are forgotten, the
 * launch counters and the HBM peak restart from now. */
int vh_serve_reset_stats(vh_ctx* ctx);

typedef struct vh_serve_stats {
    int64_t frames_done;        /* mesh-frames completed */
    int64_t requests_done;
    int64_t launches;           /* frame launches enqueued */
    double mean_batch;          /* mesh-frames per launch */
    double span_s;              /* first arrival to last request completion */
    double frames_per_second;   /* frames_done / span_s */
    double latency_p50_s, latency_p99_s, latency_max_s;   /* over completed requests */
    size_t hbm_in_use, hbm_peak;   /* context device bytes now / at most since the server opened
                                      (or since vh_serve_reset_stats) */
    int32_t meshes_resident, meshes_waiting;
} vh_serve_stats;
int vh_serve_get_stats(vh_ctx* ctx, vh_serve_stats* stats);

#ifdef __cplusplus
}
#endif
#endif /* VHPD_H */
