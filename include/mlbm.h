/* mlbm.h -- C-ABI of the MI355X (gfx950) Meshless Lattice Boltzmann library.
 *
 * The method (Strzelczyk & Matyka, arXiv 2306.01525, after Lin et al.): a
 * D2Q9 BGK lattice Boltzmann model on an irregular point cloud whose streaming
 * step is semi-Lagrangian. The population k arriving at node x_i departs from
 * the Lagrangian point x_i - e_k dx (Sec. 2.3), where it is interpolated from
 * the post-collision populations of a stencil of K nodes with precomputed
 * shape vectors of a cubic polyharmonic RBF augmented with complete
 * polynomials of degree m (Sec. 2.2, eqs. rbf_interp_set_augmented,
 * shape_vector, poly_sets). Collision is BGK (Sec. 2.1, eqs. LBM_collision,
 * feq), optionally with the body-force term of Sec. 3.
 *
 * Several clouds (n_clouds > 1) form one plan: their nodes are concatenated
 * in cloud order for every per-node input and output, and the state arrays
 * hold one [9][n_c] block per cloud. Clouds with FP32 state, a common stencil
 * rule and no walls or force are stepped by a single launch per step.
 *
 * Conventions shared by every entry point:
 *  - Memory. The caller owns every device byte (typically torch tensors). The
 *    library never allocates device memory: sizes come from the *_query calls
 *    and the caller passes buffers of at least that size. The only host
 *    allocation is the small opaque mlbm_plan object.
 *  - Pointers. "device" pointers must be addressable by the current HIP
 *    device; "host" pointers are ordinary CPU memory.
 *  - Streams. Work is enqueued on the given stream and is asynchronous unless
 *    stated. Argument checks are synchronous and return an error code.
 *  - Errors. Every call returns an mlbm_status; on failure mlbm_last_error()
 *    returns a thread-local message. No exception crosses the ABI.
 *  - Node order. Inputs and outputs that carry a per-node value use the
 *    caller's node order ("user order"). The state arrays g are internal: the
 *    library reorders nodes along a Hilbert curve and keeps g in that order.
 *  - Units. Coordinates and dx are in the cloud's units. Populations,
 *    velocities, densities and forces are in lattice units (dx = dt = 1).
 */
#ifndef MLBM_H
#define MLBM_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MLBM_OK = 0,
    MLBM_EINVAL = -1,        /* bad argument (size, parameter range, null)      */
    MLBM_ESINGULAR = -2,     /* a local RBF system is numerically singular      */
    MLBM_EHIP = -3,          /* a HIP runtime call failed                       */
    MLBM_ESMALLBUF = -4,     /* caller buffer smaller than the queried size     */
    MLBM_EUNSUPPORTED = -5   /* valid request this library does not implement   */
} mlbm_status;

enum { MLBM_FP32_DEV = 0, MLBM_FP64 = 1 };          /* mlbm_params.precision    */
enum { MLBM_STEP_VARIANTS = 10 };   /* FP32 step variants (mlbm_autotune)           */
enum { MLBM_STENCIL_PAPER = 0, MLBM_STENCIL_OWN = 1 }; /* mlbm_params.stencil_mode */

/* One point cloud (Sec. 2.2: the set X of Eulerian nodes). */
typedef struct {
    int32_t n;                  /* number of nodes, K <= n <= 268,435,455         */
    const double *x, *y;        /* device, [n] coordinates, user order            */
    const uint8_t *node_type;   /* device, [n]: 0 fluid, 1 wall; NULL = all fluid */
    double period_x, period_y;  /* > 0: periodic with that period, coordinates in
                                   [0, period); 0: open along that axis          */
    const double *normal_x, *normal_y;   /* device, [n], user order: the outward
                                   normal of the fluid domain at wall nodes (read
                                   there only); needed by bounce-back walls,
                                   otherwise may be NULL                          */
} mlbm_cloud;

/* Simulation parameters of one cloud (Algorithm 1: "simulation parameters"). */
typedef struct {
    double dx;              /* streaming distance dx_ML (Sec. 2.3), cloud units    */
    int32_t K;              /* stencil size N_L (Sec. 2.2), 6 <= K <= 48, K >= M   */
    int32_t degree;         /* polynomial augmentation degree m in {2,3,4}
                               (eq. poly_sets; m < 2 is rejected, Sec. 3)          */
    int32_t stencil_mode;   /* MLBM_STENCIL_PAPER: a departure point is
                               interpolated on the stencil of its closest node
                               (Sec. 2.3, Algorithm 1). MLBM_STENCIL_OWN: on the
                               stencil of the arriving node itself                 */
    int32_t precision;      /* MLBM_FP32_DEV: populations stored and streamed in
                               FP32 as deviations from w_k rho0; MLBM_FP64: plain
                               FP64 populations. Weights are always built in FP64 */
    double tau;             /* BGK relaxation time, > 0.5 (eq. LBM_collision)     */
    double rho0;            /* reference density (initial density when none given) */
    int32_t force_kind;     /* 0 none; 1 constant azimuthal acceleration about the
                               origin (Sec. 3), magnitude force_mag (lattice units) */
    double force_mag;
    int32_t wall_kind;      /* 0 none; 1 wall nodes (node_type 1) hold the rest
                               equilibrium feq(rho_wall, 0) after every stream and
                               receive no force; 2 bounce-back (Sec. 3): at wall
                               nodes each population entering from outside
                               (e_k . n < 0) takes the streamed value of the
                               opposite direction; wall nodes collide and are
                               forced like the others. 2 needs the normals and is
                               not available through mlbm_import_weights       */
    double rho_wall;
    int32_t with_adjoint;   /* 1: also build the transposed streaming operator
                               used by mlbm_step_adjoint (8K entries per node;
                               8 K n above 2^31 - 1 is MLBM_EUNSUPPORTED)          */
    int32_t fp32_weights_only;  /* 0: the plan keeps the FP64 shape vectors beside
                               the FP32 ones. 1 (MLBM_FP32_DEV only, else
                               MLBM_EINVAL): the FP64 ones are solved into the
                               workspace and dropped after the build, which takes
                               64 K bytes per node off the plan (about 60 % of a
                               K = 30 plan) and adds them to the workspace; then
                               mlbm_plan_export of item 3 and mlbm_interpolate
                               return MLBM_EUNSUPPORTED, and mlbm_import_weights
                               does not take it. Steps are bitwise the same     */
} mlbm_params;

typedef struct mlbm_plan mlbm_plan;  /* opaque host object; refers to the
                                        caller's plan buffer                    */

/* Read-only description of a built plan. */
typedef struct {
    int32_t n_clouds;
    int64_t n_total;          /* sum of n over clouds                             */
    int32_t K, degree, stencil_mode, precision;   /* of cloud 0                    */
    size_t state_bytes;       /* bytes of one state array g (9 populations)        */
    int64_t tile_nodes;       /* nodes per workgroup of the step kernel            */
    int32_t step_lds_bytes;   /* LDS per workgroup of the FP32 step (0: the step
                                 gathers from global memory only)                  */
    int32_t fallback_tiles;   /* tiles whose gather tables exceed the LDS caps and
                                 gather from global memory (-1: not known)         */
    int32_t variant;          /* FP32 step variant in use (mlbm_autotune)          */
} mlbm_plan_info;

/* ---- weight build (Sec. 2.2-2.3; Algorithm 1, initialisation loop) -------- */

/* Sizes of the device plan buffer and of the temporary workspace needed by
 * mlbm_build_weights for these clouds and parameters. Synchronous, no device
 * work. n_clouds >= 1; clouds and params are host arrays of n_clouds entries. */
mlbm_status mlbm_weights_query(const mlbm_cloud *clouds, const mlbm_params *params,
                               int32_t n_clouds, size_t *plan_bytes,
                               size_t *workspace_bytes);

/* Build stencils, owners and shape vectors on the GPU:
 *  1. order nodes along a Hilbert curve of a uniform cell grid;
 *  2. stencil X^L of every node: itself, then its K-1 closest nodes by
 *     (squared distance, user index), minimum image when periodic (Sec. 2.2);
 *  3. owner of every departure point x_i - e_k dx: its closest node, ties to
 *     the lower user index (paper mode), or node i (own mode) (Sec. 2.3);
 *  4. shape vectors w_L(p) = first K entries of Phi^{-1} phi_L(p) with Phi the
 *     (K+M)x(K+M) collocation matrix of r^3 plus monomials, solved in FP64 by
 *     Gaussian elimination with partial pivoting (Sec. 2.2-2.3).
 * plan_buf (device, plan_bytes) must stay allocated while the plan is used;
 * workspace (device, workspace_bytes) is free again when the stream reaches
 * the end of this call's work. *out receives a host object to release with
 * mlbm_plan_destroy. When the stream is not being captured, the call waits
 * for the build and returns MLBM_ESINGULAR if a local system was singular
 * (mlbm_last_error names the node); under capture, the status is left in the
 * device error word (mlbm_device_error). */
mlbm_status mlbm_build_weights(const mlbm_cloud *clouds, const mlbm_params *params,
                               int32_t n_clouds, void *plan_buf, size_t plan_bytes,
                               void *workspace, size_t workspace_bytes, mlbm_plan **out,
                               hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid allocation): the build of
 * mlbm_build_weights with no workspace argument. Its temporary arrays live in
 * a fixed 32 MiB array inside the library, one per GPU, held until the process
 * ends; clouds are built one after another on `stream`. That covers one cloud
 * of about 550,000 nodes (K 30, degree 4), 350,000 with the adjoint tables,
 * 16,000 with fp32_weights_only (whose FP64 shape vectors then live in it);
 * a build whose one-cloud-at-a-time workspace (compare mlbm_weights_query)
 * exceeds it returns MLBM_EUNSUPPORTED before any device work. plan_buf and
 * plan_bytes as for mlbm_build_weights (same size); the results are the same.
 * Calls on one GPU share the array, so calls whose work overlaps on that GPU
 * (other streams, other threads) race: order them. Allocates no device
 * memory; the host plan object is released by mlbm_plan_destroy. */
mlbm_status mlbm_build_weights_static(const mlbm_cloud *clouds, const mlbm_params *params,
                                      int32_t n_clouds, void *plan_buf, size_t plan_bytes,
                                      mlbm_plan **out, hipStream_t stream);

/* Test hook: a plan built from host arrays instead of the GPU build, for one
 * periodic or open cloud. x, y: host [n]; nbr: host int32 [n][K] stencils in
 * user indices (centre first); owner: host int32 [n][9] owner node per
 * direction (user indices); W: host FP64 [n][9][K] shape vectors. Node order
 * is taken as given (no reordering). Same buffer rules as mlbm_build_weights;
 * synchronous. */
mlbm_status mlbm_import_query(int32_t n, const mlbm_params *params, size_t *plan_bytes);
mlbm_status mlbm_import_weights(int32_t n, const double *x, const double *y,
                                const uint8_t *node_type, const int32_t *nbr,
                                const int32_t *owner, const double *W,
                                const mlbm_params *params, void *plan_buf,
                                size_t plan_bytes, mlbm_plan **out, hipStream_t stream);

mlbm_status mlbm_plan_get_info(const mlbm_plan *plan, mlbm_plan_info *info);

/* Copy an internal plan array to host memory (synchronous), for inspection:
 * what = 0 perm int32 [n] (internal position -> user index),
 *        1 nbr int32 [n][K] (user indices, node-major, user order),
 *        2 owner int32 [n][9] (user indices, user order),
 *        3 W FP64 [n][9][K] (user order; k = 0 is the identity; not with
 *          fp32_weights_only),
 *        4 tile descriptors int32 [ntiles][2] (|O_t|, |H_t|; 0 = global path),
 *        5 halo lists int32 [ntiles][hcap] (internal indices),
 *        6 local stencils uint32 [ntiles][ocap][ceil(K/3)]: halo positions of
 *          stencil slots 3w, 3w+1, 3w+2 in bits 0-9, 10-19, 20-29 of word w,
 *        7 local owners uint16 [8][n] (internal order; paper mode),
 *        8 capacities int32 [2] (ocap, hcap),
 *        9 adjoint tile descriptors int32 [ntiles] (|I_t|; 0 = global path),
 *       10 inverse halo lists int32 [ntiles][hcap] (internal indices),
 *       11 adjoint local columns uint32 [ceil((K+4)/3) * n64][8]: positions
 *          in I_t of entries 3w, 3w+1, 3w+2 of transposed row k-1 of node m
 *          (bits as in item 6), compacted like item 13 over triples w (node
 *          m takes part in triple w when 3w < hd(m)),
 *       12 transposed row pointers int32 [8n+1] (row (k-1)n + m),
 *       13 transposed row heads int32 [(K+4) * n64][8], n64 = n rounded up
 *          to a multiple of 64 (internal indices). Nodes are grouped by 64;
 *          hd(m) = max over the 8 rows of node m of min(length, K+4). Group g
 *          starts at unit g*64*(K+4), and its slot e = 0, 1, ... holds a
 *          block of c units, one for each node of the group with hd > e, in
 *          node order; unit entry k-1 is entry e of row k-1 of that node (m
 *          past the row end). A block of c units starting at unit u0 stores
 *          entries 0-3 of its units first and then entries 4-7: entry k-1 of
 *          its unit r is element 8 u0 + 4 ((k-1)/4 c + r) + (k-1)%4.
 * Items 4-8 describe the gather tables of the LDS-staged steps and items 9-13
 * those of the adjoint step (internal layout; 9-13 need with_adjoint).
 * Cloud `cloud`; dst_bytes must match exactly. */
mlbm_status mlbm_plan_export(const mlbm_plan *plan, int32_t cloud, int32_t what, void *dst,
                             size_t dst_bytes);

mlbm_status mlbm_plan_destroy(mlbm_plan *plan);   /* frees the host object only */

/* Change the relaxation time tau (> 0.5) of every cloud of the plan. The
 * shape vectors do not depend on tau, so nothing is rebuilt; a graph created
 * earlier is dropped (it holds the old value). Synchronous: it waits for the
 * device, and a multi-cloud plan's step descriptors are rewritten in place, so
 * no step of this plan may be in flight on another thread. */
mlbm_status mlbm_plan_set_tau(mlbm_plan *plan, double tau);

/* ---- time stepping (Algorithm 1, time loop) ------------------------------- */

/* Initial state: populations at equilibrium with the given macroscopic fields
 * (Algorithm 1; Sec. 3), then one collision, so that g holds post-collision
 * populations. rho: device FP64 [n_total] or NULL (uniform rho0); ux, uy:
 * device FP64 [n_total] or NULL (zero), user order. g: device, state_bytes. */
mlbm_status mlbm_init(const mlbm_plan *plan, const double *rho, const double *ux,
                      const double *uy, void *g, hipStream_t stream);

/* n_steps fused timesteps. Each step, per node: stream (interpolate the
 * post-collision populations at the departure points), apply the wall rule,
 * take the moments, collide (with force), write the new post-collision
 * populations. Ping-pong between g_a and g_b (device, state_bytes each);
 * *result_in_b (host) is set to 1 if the final state is in g_b, else 0. */
mlbm_status mlbm_step(const mlbm_plan *plan, void *g_a, void *g_b, int32_t n_steps,
                      int32_t *result_in_b, hipStream_t stream);

/* Density and velocity (eq. macro_var) of the pre-collision populations that
 * gave the post-collision state g (collision conserves mass and momentum; the
 * force contribution is removed). Outputs: device FP64 [n_total] each, user
 * order; any may be NULL. */
mlbm_status mlbm_moments(const mlbm_plan *plan, const void *g, double *rho, double *ux,
                         double *uy, hipStream_t stream);

/* Diagnostics: sums over all nodes (FP64, device out[4]) of
 * (u - u*)^2 + (v - v*)^2, u*^2 + v*^2, (u - u*)^2, u*^2 for the velocity of
 * state g against a target field (device FP64 [n_total], user order). The L2
 * norm of eq. L2norm is sqrt(out[2] / out[3]) for the u-component and
 * sqrt(out[0] / out[1]) for the vector. out is overwritten. */
mlbm_status mlbm_l2_sums(const mlbm_plan *plan, const void *g, const double *ux_t,
                         const double *uy_t, double *out, hipStream_t stream);

/* Interpolation alone (Sec. 4, Fig. interp_test): the plan's streaming
 * operator applied to a scalar field, in FP64 with the FP64 shape vectors:
 * out[k-1][i] = sum_j w_{i,k,j} field[stencil member j of the stencil that
 * serves departure point x_i - e_k dx], k = 1..8. field: device FP64
 * [n_total], user order; out: device FP64 [8][n_total], user order (clouds of
 * a multi-cloud plan at their offsets). MLBM_EUNSUPPORTED for a plan built
 * with fp32_weights_only, which has no FP64 shape vectors. */
mlbm_status mlbm_interpolate(const mlbm_plan *plan, const double *field, double *out,
                             hipStream_t stream);

/* Steady-state residual (Sec. 3, annular channel: runs stop when the relative
 * change of the velocity field falls below a threshold): with U = |u| of
 * state g at every node and speed (device FP64 [n_total], user order) holding
 * U of the previous check, out[0] = sum (U - U_prev)^2, out[1] = sum U^2
 * (out[2], out[3] = 0), so the residual is sqrt(out[0] / out[1]). speed is
 * overwritten with the current U (zero it before the first check). */
mlbm_status mlbm_residual(const mlbm_plan *plan, const void *g, double *speed, double *out,
                          hipStream_t stream);

/* ---- standard lattice Boltzmann (the paper's reference method) ----------------
 * D2Q9 BGK on a periodic nx x ny lattice of unit spacing and time step, with
 * streaming by an index shift (eq. LBM_streaming) and the collision of the
 * MLBM step (eqs. LBM_collision, feq). Node (ix, iy) is index iy * nx + ix;
 * the state is [9][ny][nx] post-collision populations, FP32 deviations from
 * w_k rho0 (MLBM_FP32_DEV) or plain FP64 (MLBM_FP64), caller-owned device
 * memory of 9 * nx * ny elements. Inputs and outputs are device FP64 [ny][nx]
 * (rho may be NULL for rho0, u for rest). nx * ny * 9 must fit in int32. */
mlbm_status mlbm_lbm_init(int32_t nx, int32_t ny, int32_t precision, double rho0,
                          const double *rho, const double *ux, const double *uy, void *g,
                          hipStream_t stream);
/* n_steps steps, ping-pong between g_a and g_b (distinct); *result_in_b = 1
 * when the result is in g_b. */
mlbm_status mlbm_lbm_step(int32_t nx, int32_t ny, int32_t precision, double tau, double rho0,
                          void *g_a, void *g_b, int32_t n_steps, int32_t *result_in_b,
                          hipStream_t stream);
mlbm_status mlbm_lbm_moments(int32_t nx, int32_t ny, int32_t precision, double rho0,
                             const void *g, double *rho, double *ux, double *uy,
                             hipStream_t stream);

/* ---- differentiation (no walls, no force) ----------------------------------- */

/* Forward steps that also record the pre-collision populations f^n of every
 * step n = 1..n_steps into f_rec (device, n_steps * state_bytes, in the
 * state's precision and layout). */
mlbm_status mlbm_step_record(const mlbm_plan *plan, void *g_a, void *g_b, int32_t n_steps,
                             void *f_rec, int32_t *result_in_b, hipStream_t stream);

/* Pre-collision populations f^0 = feq(rho0, u0) (the state before the first
 * collision). Same inputs and layout as mlbm_init. */
mlbm_status mlbm_init_f(const mlbm_plan *plan, const double *rho, const double *ux,
                        const double *uy, void *f, hipStream_t stream);

/* Collision only: g = C(f) for a pre-collision state f (same layout), so a
 * recorded or checkpointed f can restart the post-collision time loop. */
mlbm_status mlbm_collide(const mlbm_plan *plan, const void *f, void *g, hipStream_t stream);

/* Seed of the adjoint for J = 1/2 sum_i |u_i(f_T) - u*_i|^2: lamf_T = dJ/df_T.
 * f_T: pre-collision state (device, state precision and layout); ux_t, uy_t:
 * device FP64 [n_total] user order; lamf_T: device, state_bytes, adjoint
 * populations in the state precision and layout; J: device FP64 [1],
 * overwritten. Plans with walls or a body force return MLBM_EUNSUPPORTED. */
mlbm_status mlbm_loss_seed(const mlbm_plan *plan, const void *f_T, const double *ux_t,
                           const double *uy_t, void *lamf_T, double *J,
                           hipStream_t stream);

/* One reversed step. The forward step maps f^n to f^{n+1} = S(C(f^n)) (C
 * collision, S streaming). Given the adjoint lamf_next of f^{n+1} and the
 * recorded pre-collision f^n, computes lamf_n = C'(f^n)^T S^T lamf_next: a
 * gather over the transposed streaming weights (built when the plan was made
 * with_adjoint), then the transposed BGK Jacobian at f^n. Adds this step's
 * dJ/dtau = (S^T lamf_next) . dC/dtau (f^n) into dJ_dtau (device FP64 [1],
 * accumulated). lamf_*: device, state_bytes, state precision and layout. */
mlbm_status mlbm_step_adjoint(const mlbm_plan *plan, const void *f_n, const void *lamf_next,
                              void *lamf_n, double *dJ_dtau, hipStream_t stream);

/* dJ/du0 = (d feq(rho0, u0) / d u0)^T lamf_0, with f^0 = feq(rho0, u0) the
 * state before the first collision. u0x, u0y: device FP64 [n_total], user
 * order (NULL = 0); outputs device FP64 [n_total] each, user order. */
mlbm_status mlbm_init_adjoint(const mlbm_plan *plan, const double *u0x, const double *u0y,
                              const void *lamf_0, double *dJ_du0x, double *dJ_du0y,
                              hipStream_t stream);

/* ---- tuning --------------------------------------------------------------- */

/* Autotuner of the FP32 step: times every kernel variant (the unroll depth
 * of the stencil loop, non-temporal weight loads, one or two lanes per node)
 * for n_steps steps each, after one warm-up step, on this plan's own cloud,
 * and keeps the fastest for every later step and graph. ms_out (host, may be
 * NULL, room for MLBM_STEP_VARIANTS floats) receives the measured milliseconds
 * per step of each variant, *n_variants (host, may be NULL) their count. The contents of
 * g_a and g_b are advanced (start again from mlbm_init afterwards). Synchronous. FP64 plans have a single variant. */
mlbm_status mlbm_autotune(mlbm_plan *plan, void *g_a, void *g_b, int32_t n_steps,
                          float *ms_out, int32_t *n_variants, hipStream_t stream);

/* The whole batched workload as one HIP graph: captures, on `stream` (not the
 * default stream), the weight build of every cloud (mlbm_build_weights), the
 * initial state from rho/ux/uy into g_a (mlbm_init) and n_steps steps on
 * (g_a, g_b) (mlbm_step) with FP32 step variant `variant`. Nothing runs until
 * mlbm_graph_launch; each launch rebuilds the weights and restarts from the
 * initial state. Buffers as for those calls; the workspace and the inputs must
 * stay allocated while the graph is used. The step LDS size is chosen before
 * the tables exist (no size read-back under capture): 40 KiB for FP32 plans up
 * to K = 30, where a tile whose tables need more gathers from global memory
 * instead (same results, slower), else the capacity bound. A singular system
 * is reported through mlbm_device_error after a launch. */
mlbm_status mlbm_build_graph(const mlbm_cloud *clouds, const mlbm_params *params,
                             int32_t n_clouds, void *plan_buf, size_t plan_bytes,
                             void *workspace, size_t workspace_bytes, const double *rho,
                             const double *ux, const double *uy, void *g_a, void *g_b,
                             int32_t n_steps, int32_t variant, mlbm_plan **out,
                             hipStream_t stream);

/* Select an FP32 step variant by index (0 = default); drops a created graph. */
mlbm_status mlbm_plan_set_variant(mlbm_plan *plan, int32_t variant);

/* ---- graphs ------------------------------------------------------------- */

/* Capture n_steps steps on (g_a, g_b) into a HIP graph owned by the plan
 * (replaces a previous one). mlbm_graph_launch replays it on `stream`.
 * The graph is destroyed by mlbm_plan_destroy. */
mlbm_status mlbm_graph_create(mlbm_plan *plan, void *g_a, void *g_b, int32_t n_steps,
                              hipStream_t stream);
mlbm_status mlbm_graph_launch(mlbm_plan *plan, hipStream_t stream);

/* ---- errors --------------------------------------------------------------- */

const char *mlbm_last_error(void);

/* Conditions the kernels record in a plan's sticky device error words (bits;
 * several may be set). They never stop a kernel: a diverging run finishes its
 * steps and the caller decides what to do. */
enum {
    MLBM_DEVERR_SINGULAR = 1,   /* a local RBF system was numerically singular
                                   (mlbm_build_weights, mostly under capture)      */
    MLBM_DEVERR_INDEX = 2,      /* a gather table of the plan held a node index
                                   outside the cloud; that gather read node 0
                                   instead (the plan buffer was overwritten)       */
    MLBM_DEVERR_NONFINITE = 4,  /* a node's density or velocity was NaN or Inf     */
    MLBM_DEVERR_SPEED = 8       /* a node's speed exceeded 0.3 (lattice units;
                                   Mach 0.52): the run is diverging, as the method
                                   does for some stencils and spacings (Sec. 3)    */
};

/* The plan's device error bits (MLBM_DEVERR_*), read synchronously (waits for
 * the device): 0 none, -1 if the read failed. Set by the build (singular
 * systems), by every step (non-finite or too fast nodes, out-of-range halo
 * indices) and by mlbm_moments, mlbm_l2_sums and mlbm_residual (non-finite or
 * too fast nodes). */
int32_t mlbm_device_error(const mlbm_plan *plan);

/* The nodes behind the bits, synchronous: *singular_node = user index of the
 * first node (lowest index) whose local system was singular, and
 * *diverged_node = the lowest user index reported non-finite or too fast; -1
 * where none is known. Either pointer may be NULL (host). */
mlbm_status mlbm_device_error_nodes(const mlbm_plan *plan, int32_t *singular_node,
                                    int32_t *diverged_node);

/* Reset the device error words to "none" (enqueued on `stream`; kernels only,
 * so it may be captured). */
mlbm_status mlbm_device_error_clear(mlbm_plan *plan, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* MLBM_H */
