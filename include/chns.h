/*
 * chns.h - C ABI of libchns: the matrix-free hot path of the projection-based
 * semi-implicit Cahn-Hilliard Navier-Stokes (CHNS) solver on adaptive
 * 2:1-balanced octrees, for one AMD MI355X (gfx950).
 *
 * Conventions for every call:
 *   - Return value: CHNS_OK (0) or a negative error code; no call aborts or
 *     throws across the ABI.  chns_last_error() returns a thread-local message.
 *   - Handles (chns_mesh, chns_ctx) are opaque, owned by the library and freed
 *     with their *_destroy call.
 *   - Vector arguments named x, y, b, phi ... are caller-owned, contiguous
 *     DEVICE memory on the context's device, in the mesh's independent-node
 *     order (chns_mesh_node_coords).  The library never keeps such a pointer
 *     after the call returns.  FP64 vectors are double*, FP32 vectors float*.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Calls marked
 *     "async" only enqueue work on it; the others synchronise it before
 *     returning.
 *   - A context must not be used by two threads at once.
 *
 * Citations refer to the paper "A projection-based, semi-implicit
 * time-stepping approach for the Cahn-Hilliard Navier-Stokes equations on
 * adaptive octree meshes" (Khanwale et al.): sections, definitions and
 * equations by their names in the paper.
 */
#ifndef CHNS_H
#define CHNS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  CHNS_OK = 0,
  CHNS_EINVAL = -1,  /* bad argument, shape or state combination            */
  CHNS_ENOMEM = -2,  /* host or device allocation failed                     */
  CHNS_EHIP = -3,    /* a HIP runtime call failed (message has the HIP error) */
  CHNS_ENOCONV = -4, /* solver stopped at max_it; outputs hold the last iterate */
  CHNS_ESTATE = -5   /* call made before a required earlier call            */
};

/* ------------------------------------------------------------------ mesh */

/* Refinement rules (paper Sec. 4.2: top-down refinement by a user predicate
 * on the octant, followed by 2:1 balancing).                                */
enum {
  CHNS_RULE_UNIFORM = 0,           /* every leaf at max_level                  */
  CHNS_RULE_SPHERE_BAND = 1,       /* refine to max_level every octant meeting
                                      radius-band <= |x - centre| <= radius+band;
                                      min_level everywhere                     */
  CHNS_RULE_MULTI_SPHERE_BAND = 2, /* union over n_spheres of the above        */
  CHNS_RULE_CALLBACK = 3           /* refine while refine(anchor, level, user) */
};

typedef struct chns_mesh_spec {
  int dim;        /* 2 or 3                                                   */
  int min_level;  /* every leaf is at least this deep                         */
  int max_level;  /* no leaf is deeper; 1 <= max_level <= 16                  */
  int rule;       /* CHNS_RULE_*                                              */
  int n_spheres;  /* number of centres/radii (band rules)                     */
  const double* centres; /* host, n_spheres * dim, unit-domain coordinates    */
  const double* radii;   /* host, n_spheres                                   */
  double band;           /* half width of the refined shell                   */
  /* CALLBACK rule: anchor in integer units of 2^-max_level (unused entries 0);
   * return nonzero to refine the octant further.                            */
  int (*refine)(const int64_t anchor[3], int level, void* user);
  void* user;
  /* largest brick edge (8, 4, 2 or 1 leaves); 0 = automatic: the largest
   * edge that still gives >= 1024 bricks, so small meshes keep the GPU busy */
  int brick_max;
  /* Incomplete (carved) octree (paper Sec. 4: traversals visit only the
   * octants that exist, so the domain can be a union of octants; Sec. 5.4
   * runs in a 1 x 8 x 1 box): carve_level = 0 keeps the whole unit cube;
   * otherwise only the octants inside the box [0, extent[d] 2^-carve_level]
   * per direction d exist (extent[2] unused in 2D).  Needs
   * 1 <= carve_level <= min_level and 1 <= extent[d] <= 2^carve_level.  The
   * velocity walls are the faces of the box; phi, mu and the pressure keep
   * natural conditions there.                                              */
  int carve_level;
  int32_t extent[3];
} chns_mesh_spec;

typedef struct chns_mesh chns_mesh;

typedef struct chns_mesh_info {
  int dim, max_level;
  int node_order;        /* 0 = lexicographic (x fastest; uniform meshes),
                            1 = Morton, 2 = blocked: aligned 8^d blocks of
                            the finest grid in Morton order, lexicographic
                            (x fastest) inside a block (other meshes)       */
  int uniform;           /* 1 if the mesh is the whole cube with every leaf at
                            max_level                                         */
  int64_t n_elems;       /* leaves                                           */
  int64_t n_nodes;       /* independent nodes = vector length                */
  int64_t n_hanging;     /* hanging (constrained) nodes                      */
  int64_t n_bricks[4];   /* bricks of 8^d, 4^d, 2^d and single elements      */
  int64_t elems_in_bricks[4];
  int64_t n_slots;       /* brick-boundary partial sums per field            */
  int64_t n_shared;      /* nodes completed by the deterministic combine pass */
  int n_colors;          /* node colours used to probe the exact diagonal    */
  int64_t level_counts[17];
  int32_t box[3];        /* domain box in units of 2^-max_level (2^max_level
                            per direction for the whole cube)                 */
} chns_mesh_info;

/* Build a 2:1 vertex-balanced octree on the unit cube/square, enumerate its
 * independent nodes and hanging-node constraints (paper Sec. 4.2-4.3), and
 * group its leaves into bricks.  Host-only: needs no GPU.  EINVAL on a bad
 * spec; *out is owned by the caller and freed with chns_mesh_destroy.      */
int chns_octree_build(const chns_mesh_spec* spec, chns_mesh** out);
int chns_mesh_destroy(chns_mesh* mesh);
int chns_mesh_info_get(const chns_mesh* mesh, chns_mesh_info* out);
/* Integer coordinates (units 2^-max_level) of the independent nodes in vector
 * order: host buffer of n_nodes * dim int64.                                */
int chns_mesh_node_coords(const chns_mesh* mesh, int64_t* ijk);
/* Leaves in Morton order: host buffers level[n_elems], anchor[n_elems*dim]. */
int chns_mesh_leaves(const chns_mesh* mesh, int32_t* level, int64_t* anchor);
/* Hanging nodes: coords[n_hanging*dim] and parent indices parents[n_hanging*4]
 * (independent-node indices, -1 padded), host buffers.                     */
int chns_mesh_hanging(const chns_mesh* mesh, int64_t* coords, int32_t* parents);

/* ------------------------------------------------------------- remeshing */

/* Remeshing by the phase field (paper: adaptive refinement of the interface
 * region |phi| <= 0.95, Sec. 4.2 top-down refinement by a predicate, and the
 * scaling section's refine/coarsen as the interface moves): a new octree of
 * the same dimension and max_level whose octants are refined to max_level
 * wherever the nodal values of `phi` inside the octant's half-open box (the
 * old mesh's independent nodes, and its hanging nodes at the mean of their
 * parents) span a range that meets [-threshold, threshold], and to
 * min_level elsewhere; 2:1 balanced like chns_octree_build.  phi: host,
 * old n_nodes doubles in vector order.  brick_max as in chns_mesh_spec.
 * Host-only.  EINVAL on a bad argument; *out is owned by the caller.       */
int chns_mesh_remesh(const chns_mesh* old, const double* phi, int min_level, double threshold, int brick_max,
                     chns_mesh** out);

/* Intergrid transfer of nodal fields from mesh `from` to mesh `to` (same
 * dimension and max_level; paper Sec. 4, traversal-based intergrid
 * transfers): every node of `to` takes the value of the Q1 field of `from`
 * (hanging constraints included) at its position.  This copies at
 * coincident nodes, interpolates the shape functions into refined leaves and
 * takes the coinciding fine values for coarsened ones; with nested Q1
 * spaces it equals any sequence of one-level transfers.  Not conservative.
 * create: host-only, builds the CSR (rows: nodes of `to`, columns: nodes of
 * `from`); info / matrix copy it to host buffers (ptr rows + 1, col and val
 * nnz); apply: y (rows * n_fields, device) = the transfer of x (cols *
 * n_fields, device), field-blocked, on `stream`; x and y must not alias; the
 * first apply uploads the CSR to the current device (synchronously), later
 * applies on another device are EINVAL.  Async.  EINVAL for meshes of
 * different dimension or max_level, null pointers or n_fields < 1.  *out
 * is owned by the caller and freed, with its device copy, by
 * chns_transfer_destroy.                                                   */
typedef struct chns_transfer chns_transfer;
int chns_transfer_create(const chns_mesh* from, const chns_mesh* to, chns_transfer** out);
int chns_transfer_info(const chns_transfer* t, int64_t* rows, int64_t* cols, int64_t* nnz);
int chns_transfer_matrix(const chns_transfer* t, int32_t* ptr, int32_t* col, double* val);
int chns_transfer_apply(chns_transfer* t, int n_fields, const double* x, double* y, void* stream);
int chns_transfer_destroy(chns_transfer* t);

/* --------------------------------------------------------------- context */

/* Non-dimensional parameters (paper Sec. 2 and its non-dimensionalisation
 * subsection).  Pe <= 0 selects 1/Pe = 3 Cn^2.  C_I <= 0 selects 6.        */
typedef struct chns_params {
  double Re, We, Cn, Pe, Fr;
  double rho_plus, rho_minus;  /* specific densities; rho(phi) = alpha phi + beta */
  double eta_plus, eta_minus;  /* specific viscosities                           */
  double dt;                   /* time step                                      */
  double C_I;                  /* VMS constant                                   */
  int gravity_axis;            /* gravity is -e_axis (default 1 = y)             */
} chns_params;

typedef struct chns_ctx chns_ctx;

/* Upload the mesh to the current HIP device and allocate work buffers.
 * The mesh must outlive the context.                                       */
int chns_context_create(chns_mesh* mesh, const chns_params* params, chns_ctx** out);
int chns_context_destroy(chns_ctx* ctx);

/* Phase field used by the variable-coefficient operators: the context keeps
 * its own FP64 and FP32 copies of phi~ = (phi + phi_prev)/2, or of phi when
 * phi_prev is NULL (paper Sec. 3, time averages).  Async.                   */
int chns_set_phase_field(chns_ctx* ctx, const double* phi, const double* phi_prev, void* stream);

/* ------------------------------------------------------------- operators */

enum {
  CHNS_OP_PRESSURE = 0,    /* y = A x,  A = -div((1/rho(phi*~)) grad .): pressure
                              Poisson of Def. 2 / VMS pressure Poisson, natural BCs;
                              1 field                                           */
  CHNS_OP_MOMENTUM = 1,    /* VMS velocity prediction (Def. 3), dim fields,
                              component-blocked; wall rows are identity        */
  CHNS_OP_CH_JACOBIAN = 2, /* Newton Jacobian of the discrete CH system (Def. 6):
                              2 fields (phi block then mu block)                */
  CHNS_OP_MASS_RHO = 3,    /* (w, rho(phi*~) u): velocity update (Def. 5), dim
                              fields, wall rows identity                        */
  CHNS_OP_MASS = 4,        /* (q, u): plain Q1 mass, 1 field                    */
  CHNS_OP_MOMENTUM_SCALAR = 5 /* (w, rho(phi*~)/dt u) + (grad w, eta(phi*~)/(2 Re)
                              grad u): the mass and viscous part of Def. 3 for one
                              velocity component, natural BCs (no wall rows); the
                              operator of the momentum multigrid preconditioner;
                              1 field, uses the phase field                     */
};
enum { CHNS_FP64 = 0, CHNS_FP32 = 1 };

/* y = Op x, matrix-free: per leaf, gather (with hanging-node interpolation),
 * 2-point Gauss quadrature, and a conflict-free deterministic scatter-add
 * (transpose interpolation).  x and y: device, n_fields * n_nodes of the
 * precision's type; x and y must not alias.  Every operator is available in
 * CHNS_FP64 and CHNS_FP32; in FP32 the arithmetic and the fields are single
 * precision (the phase field kept as 1 + phi so that rho(phi) keeps its
 * relative accuracy near phi = -1; MOMENTUM and CH_JACOBIAN use FP32 copies
 * of their coefficient fields, made on the first FP32 apply after each
 * chns_set_coefficients).  ESTATE before chns_set_phase_field (PRESSURE,
 * MASS_RHO, MOMENTUM_SCALAR) or chns_set_coefficients (MOMENTUM,
 * CH_JACOBIAN).  Async.                                                     */
int chns_apply_operator(chns_ctx* ctx, int op, int prec, const void* x, void* y, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * y = Op x as chns_apply_operator, same kernels and bitwise the same result,
 * but the brick-boundary partial sums live in a static per-GPU scratch array
 * of 32 MiB (held by each GPU the library runs on until the process ends)
 * instead of the context's slot buffer.  The call allocates nothing.
 * Arguments as chns_apply_operator; the current device must be the
 * context's.  EINVAL when the mesh needs more scratch than 32 MiB for this
 * operator and precision (fields * brick-boundary slots * element size; a
 * 128^3 mesh of 8^3 bricks has 1.58 M slots and fits for every operator but
 * the three-field FP64 momentum operator), or while profiling is enabled.  Every call on one GPU
 * (any context, any stream) uses the same array and overwrites it: calls
 * that overlap in time on one GPU race and give wrong results; calls ordered
 * on one stream, or separated by synchronisation, are safe.  Async.        */
int chns_apply_operator_noalloc(chns_ctx* ctx, int op, int prec, const void* x, void* y, void* stream);

/* Exact diagonal of the constrained operator diag(P^T (sum_e K_e) P),
 * including the cross terms that hanging nodes create.  d: device,
 * n_fields * n_nodes.  Async.                                              */
int chns_operator_diagonal(chns_ctx* ctx, int op, int prec, void* d, void* stream);

/* ---------------------------------------------------------------- solves */

enum { CHNS_PC_JACOBI = 0, CHNS_PC_GMG = 1, CHNS_PC_LEARNED = 2, CHNS_PC_NONE = 3 };
/* MIXED_IR: FP64 iterative refinement, r = b - A x in FP64, each inner CG
 * (FP32 operator, vectors and preconditioner; FP64 dot products) solves
 * A d = r / |r| to inner_rtol from a fresh start, then x += |r| d.
 * MIXED_RU: the same refinement steps, but each inner CG continues the
 * previous one's search direction (residual replacement, as in reliable-
 * update CG): p = z + beta p with beta = (r.z)_new / (r.z)_old of the
 * unnormalised residuals, so the Krylov process is not restarted when the
 * FP64 residual replaces the FP32 one (flexible CG with the learned
 * preconditioner: the Polak-Ribiere beta, z.(r_new - r_prev) / (r.z)_prev,
 * with the previous inner system's vectors rescaled to the new one).       */
enum { CHNS_MODE_FP64 = 0, CHNS_MODE_MIXED_IR = 1, CHNS_MODE_MIXED_RU = 2 };

typedef struct chns_solve_opts {
  double rtol;        /* stop when |b - A x|_2 / |b|_2 <= rtol (FP64); default 1e-8 */
  int max_it;         /* Krylov iterations (inner ones in MIXED_IR); default 20000   */
  int pc;             /* CHNS_PC_*                                                   */
  int mode;           /* CHNS_MODE_*                                                 */
  double inner_rtol;  /* MIXED_IR inner tolerance; default 1e-4.  MIXED_RU: the
                         factor by which the FP32 residual falls between two FP64
                         replacements; about 1e-2 (below ~1e-3 FP32 rounding piles
                         up in the continued directions and convergence stalls)    */
  int check_every;    /* host convergence poll period in iterations; default 16      */
  int max_outer;      /* MIXED_IR / MIXED_RU refinement steps; default 30            */
  int no_graphs;      /* 1: launch every kernel eagerly instead of replaying one HIP
                         graph per Krylov iteration (same arithmetic, same result)  */
  int learned_every;  /* CHNS_PC_LEARNED: 0 = network preconditioner in every
                         flexible-CG iteration (abandoned for Jacobi after 400
                         iterations without convergence); k > 0 = network on r_0
                         and after every k-th iteration, Jacobi after the others */
} chns_solve_opts;

typedef struct chns_solve_stats {
  int iterations;        /* total Krylov iterations (all inner ones in MIXED_IR)  */
  int outer_iterations;  /* FP64 refinement steps (MIXED_IR), else 1               */
  double rel_residual;   /* FP64 true |b - A x|/|b| at exit, recomputed            */
  double ms_setup;       /* diagonal / hierarchy / network set-up                  */
  double ms_solve;       /* iterations + final residual                            */
  int fallback;          /* 1 if the learned preconditioner was abandoned          */
} chns_solve_stats;

/* Solve the pressure Poisson system A x = b for the current phase field.
 * A is singular (constants); b is projected to 1^T b = 0 first and x is
 * returned with 1^T x = 0.  b, x: device FP64, n_nodes; x holds x0 on entry
 * (use zeros for the standard start).  Synchronises `stream`.  ENOCONV if
 * rtol was not reached; x and stats then describe the last iterate.  A CG
 * breakdown (p.Ap <= 0 or r.z <= 0, e.g. a preconditioner output of zero)
 * ends the iteration at the last iterate: with the learned preconditioner
 * the solve then continues with Jacobi (stats->fallback = 1), otherwise it
 * is ENOCONV.  EINVAL, with stats filled (0 iterations, rel_residual NaN)
 * and x unchanged, when the phase field given to chns_set_phase_field or b
 * holds a NaN or an infinity.                                             */
int chns_solve_pressure(chns_ctx* ctx, const double* b, double* x, const chns_solve_opts* opts,
                        chns_solve_stats* stats, void* stream);

/* ------------------------------------------------- CHNS forms and stepping */

/* Coefficient fields of the CHNS operators (device FP64, copied into the
 * context; the caller keeps ownership).  Vectors are component-blocked
 * (dim * n_nodes).  Async.
 *   CHNS_OP_MOMENTUM:    fields = {phi~, mu~, u^}: time-averaged phase field
 *                        and chemical potential, extrapolated velocity
 *                        u^ = (3 u^k - u^{k-1})/2 (Sec. 3, Def. 3; the
 *                        mixture current J is built from grad mu~)
 *   CHNS_OP_CH_JACOBIAN: fields = {phi^{k+1} (Newton iterate), phi^k, u~}
 *                        (Def. 6); the Jacobian reads the two phase fields
 *                        only through their average, which the context
 *                        stores in their place
 * EINVAL for any other op.                                                 */
int chns_set_coefficients(chns_ctx* ctx, int op, const double* const* fields, void* stream);

/* Right-hand sides, residuals and energy densities assembled matrix-free with
 * the same gather / quadrature / conflict-free scatter as the operators.    */
enum {
  CHNS_FORM_CH_RESIDUAL = 0, /* fields {x = [phi^{k+1}; mu^{k+1}] (2n), phi^k, mu^k, u~ (dim n)}
                                -> (R_phi, R_mu), 2n (Def. 6)                   */
  CHNS_FORM_VP_RHS = 1,      /* fields {phi~, mu~, u^, u^k, p^k} -> dim n, wall rows 0
                                (Def. 3 right-hand side incl. gravity, Korteweg
                                and the known part of the VMS fine scales; no
                                body force: see chns_step_opts.force_v)        */
  CHNS_FORM_PP_RHS = 2,      /* fields {.. as VP_RHS .., v} -> n (Def. 4, including
                                the fine-scale term of the predicted velocity)  */
  CHNS_FORM_VU_RHS = 3,      /* fields {.. as PP_RHS .., p^{k+1}} -> dim n, wall rows 0
                                (Def. 5)                                        */
  CHNS_FORM_ENERGY = 4       /* fields {phi, u} -> n: each leaf's free energy
                                (kinetic + mixing + gravitational, Sec. 2) split
                                equally over its corners; the sum is the total */
};
int chns_assemble(chns_ctx* ctx, int form, const double* const* fields, double* out, void* stream);

/* mu^0 as the L2 projection (q, mu) = (q, psi'(phi)) + Cn^2 (grad q, grad phi)
 * (the paper does not state the initial chemical potential).  phi, mu:
 * device FP64, n_nodes.  Synchronises `stream`.                             */
int chns_initial_mu(chns_ctx* ctx, const double* phi, double* mu, void* stream);

/* State of the time stepper: caller-owned device FP64 arrays, updated in
 * place from step k to k + 1.  u and u_prev: dim * n_nodes (component
 * blocked; zero on the walls); p, phi, mu: n_nodes.                        */
typedef struct chns_state {
  double* u;
  double* u_prev;
  double* p;
  double* phi;
  double* mu;
} chns_state;

typedef struct chns_step_opts {
  int blocks;          /* passes of CH -> VP -> PP -> VU per step; default 2     */
  double newton_rtol;  /* Newton stop |R| <= max(newton_rtol |R0|, newton_atol); 1e-8 */
  double newton_atol;  /* default 1e-12                                          */
  int max_newton;      /* default 20                                             */
  double lin_rtol;     /* relative residual of every linear solve; default 1e-8 */
  int max_it;          /* iteration cap of each linear solve; default 5000      */
  int restart;         /* GMRES restart length, 1..128; default 64              */
  int pp_pc;           /* CHNS_PC_JACOBI (default) or CHNS_PC_GMG                */
  int pp_mode;         /* CHNS_MODE_FP64 (default), _MIXED_IR or _MIXED_RU        */
  int no_graphs;       /* 1: no HIP graph replay of Krylov iterations           */
  int ch_pc;           /* preconditioner of the CH Newton GMRES: CHNS_CH_PC_BLOCK_JACOBI
                        * (default: 2x2 node blocks of the Jacobian) or
                        * CHNS_CH_PC_SCHUR_GMG (block lower-triangular with a
                        * multigrid Schur-complement approximation; needs a
                        * mesh of max_level >= 2)                              */
  int vp_pc;           /* preconditioner of the velocity-prediction GMRES:
                        * CHNS_VP_PC_JACOBI (default) or CHNS_VP_PC_GMG (one
                        * V-cycle of CHNS_OP_MOMENTUM_SCALAR per velocity
                        * component on the interior rows, identity on the wall
                        * rows; needs a mesh of max_level >= 2)                 */
  /* Body forces for manufactured solutions (paper Sec. 5.1: the residual of
   * the continuous equations for a prescribed solution is added as a body
   * force), nodal values at the step's mid time t^k + dt/2, device FP64,
   * each nullable (NULL = zero): force_v (dim * n, component-blocked) is the
   * known right-hand side of the momentum equation, (w, f_v) in the
   * velocity prediction and -f_v inside the fine-scale residual R_m of the
   * prediction, the pressure Poisson and the velocity update; force_phi (n)
   * enters the phase-field equation as -(q, f_phi), force_mu (n) the
   * chemical-potential equation as +(q, f_mu).                            */
  const double* force_v;
  const double* force_phi;
  const double* force_mu;
} chns_step_opts;

enum { CHNS_CH_PC_BLOCK_JACOBI = 0, CHNS_CH_PC_SCHUR_GMG = 1 };
enum { CHNS_VP_PC_JACOBI = 0, CHNS_VP_PC_GMG = 1 };

typedef struct chns_step_stats {
  int newton_iterations[4]; /* per block                                        */
  int ch_iterations;        /* GMRES iterations of all Newton corrections      */
  int vp_iterations;        /* GMRES iterations of the velocity prediction    */
  int pp_iterations;        /* CG iterations of the pressure Poisson solves   */
  int vu_iterations;        /* CG iterations of the velocity update          */
  double ch_residual;       /* final |R| of the last Newton iteration        */
  double mass;              /* integral of phi^{k+1}                          */
  double energy;            /* total energy of the new state                  */
  double ms;                /* wall time of the call                          */
} chns_step_stats;

/* One projection time step (paper Sec. 3 and its flowchart): `blocks` passes
 * of Newton on the Cahn-Hilliard system (GMRES with 2x2 node-block Jacobi, or
 * with opts->ch_pc = CHNS_CH_PC_SCHUR_GMG the block lower-triangular
 * preconditioner whose Schur complement ~ (1/dt)(M + sqrt(b) K) M_L^-1
 * (M + sqrt(b) K), b = dt Cn / (2 Pe), is applied with two multigrid V-cycles;
 * the multigrid hierarchy is shared with the pressure solve and set up again
 * for it),
 * velocity prediction (GMRES with Jacobi, or with opts->vp_pc =
 * CHNS_VP_PC_GMG multigrid V-cycles of the scalar mass + viscous operator of
 * each component, hierarchy set up for it and again for the pressure solve),
 * pressure Poisson (CG) and velocity
 * update (CG on the rho-weighted mass matrix), then
 * (u_prev, u, p, phi, mu) <- (u^k, u^{k+1}, p^{k+1}, phi^{k+1}, mu^{k+1}).
 * Synchronises `stream`.  On return the context's phase field is phi~ of
 * the last block (later pressure applies and solves use it).  ENOCONV if a
 * solve or Newton stalls, or if a residual is not finite (NaN or infinity in
 * the state); the state is then left at step k, and the context's phase
 * field is marked unset (pressure applies and solves return ESTATE until
 * chns_set_phase_field).                                                   */
int chns_advance_step(chns_ctx* ctx, chns_state* state, const chns_step_opts* opts, chns_step_stats* stats,
                      void* stream);

/* ------------------------------------------------ learned preconditioner */

/* A 3D U-Net on the node grid of a uniform 3D mesh (4 levels, channels
 * 16/32/48/64, two 3x3x3 conv + ReLU per level and side, 2x2x2 average
 * pooling, nearest upsampling with skip concatenation, 1x1x1 output conv),
 * bfloat16 weights and activations with FP32 accumulation (MFMA), FP32
 * master weights and Adam.  Inputs per voxel: log(1/rho(phi*)) normalised by
 * log(rho+/rho-), and r / rms(r).  N(r) = rms(r) K Net(...).  As the
 * preconditioner CHNS_PC_LEARNED of chns_solve_pressure (flexible CG): with
 * damping omega = 0, z = N(r); with omega > 0 the network is the coarse
 * correction between two damped-Jacobi sweeps, z1 = omega D^-1 r,
 * r1 = r - A z1, n = N(r1), z2 = z1 + beta n with the A-norm-optimal step
 * beta = n.r1 / n.A n along n (either sign; 0 if n.A n <= 0),
 * z = z2 + omega D^-1 (r - A z2); then 1^T z = 0.
 * On an adaptive 3D octree of the whole cube (max_level >= 7) the network
 * sees the uniform level-7 node grid (129^3 points): N(r) = P Net(R r) with
 * P the Q1 interpolation of grid fields at the mesh's nodes, R = P^T, and
 * phi~ sampled at the grid points by the mesh's Q1 field; the transfers are
 * built on the host at the first learned solve of a context (EINVAL for 2D
 * or carved meshes, or max_level < 7).  Training and chns_pc_forward need a
 * uniform 3D mesh.
 * The paper preconditions with algebraic multigrid; this network is an
 * addition of this library.  Weights belong to the context.               */

/* Deterministic He initialisation from `seed`; out_scale is K >= 0 (K = 0
 * makes the network's output zero, which flexible CG detects as a breakdown:
 * the solve then falls back to Jacobi), smooth_omega the damping
 * (0 <= omega < 2).  EINVAL otherwise.  Async.                             */
int chns_pc_init(chns_ctx* ctx, uint64_t seed, float out_scale, float smooth_omega, void* stream);
/* Weight blob: "CHNSUNET", u32 version (1 or 2), u32 layers (14), f32 K,
 * [version 2: f32 omega], then per layer u32 ci, u32 co, f32 W[27][ci][co]
 * (tap = 9(dz+1) + 3(dy+1) + dx+1), then u32 16, f32 w_out[16]; little
 * endian; version 1 means omega = 0.  chns_pc_save writes version 2.
 * EINVAL on any mismatch.                                                  */
int chns_pc_load(chns_ctx* ctx, const void* blob, size_t n, void* stream);
/* *n = blob size; writes the blob when blob != NULL and cap >= *n.         */
int chns_pc_save(chns_ctx* ctx, void* blob, size_t cap, size_t* n);
/* Number of FP32 parameters (the blob's weights in order).                 */
int chns_pc_param_count(chns_ctx* ctx, size_t* n);
/* Gradient of the last chns_pc_train_step's mean loss, in parameter order,
 * host buffer of exactly chns_pc_param_count floats.                       */
int chns_pc_gradients(chns_ctx* ctx, float* host, size_t n);

/* Network output on a crop of the node grid: crop^3 voxels (crop a multiple
 * of 8) starting at node `origin` (x, y, z; host) with axes mirrored inside
 * the crop by the bits of `flip`; voxels beyond the grid are zero input.
 * phi, r: device FP64 node vectors; out: device FP32, crop^3 (x fastest).
 * Async.                                                                   */
int chns_pc_forward(chns_ctx* ctx, const double* phi, const double* r, const int32_t* origin, int flip, int crop,
                    float* out, void* stream);

/* One training step over n samples (phase field, residual r, error e with
 * A e = r: the exact solution minus an iterate), averaged; gradients by
 * backpropagation (MFMA input and weight gradients), then one Adam step
 * (b1 0.9, b2 0.999, eps 1e-8) when lr > 0.  Objectives:
 *   CHNS_PC_OBJ_ANORM: on the full node grid, the preconditioner output
 *     z = rms(r) K Net(...) is scored by the A-norm error
 *     (e - z)^T A (e - z) / e^T r (1 for z = 0); its gradient
 *     2 (A z - r) / e^T r takes one pressure-operator apply with the
 *     sample's phase field (which the call leaves set in the context);
 *     origin, flip and crop are unused;
 *   CHNS_PC_OBJ_CROP_MSE: on the crop (origin, flip, crop) the output is
 *     compared with e / (rms(r) K) by the mean squared error over the voxels
 *     inside the grid.
 * EINVAL when the output scale K is 0.  Synchronises `stream`.             */
enum { CHNS_PC_OBJ_CROP_MSE = 0, CHNS_PC_OBJ_ANORM = 1 };
typedef struct chns_pc_batch {
  int n;                      /* samples                                      */
  const double* const* phi;   /* host array of n device pointers (n_nodes)   */
  const double* const* r;     /* residuals                                   */
  const double* const* e;     /* errors                                      */
  const int32_t* origin;      /* host, 3 per sample (x, y, z) in nodes       */
  const int32_t* flip;        /* host, per sample; may be NULL               */
  int crop;                   /* crop edge, multiple of 8                    */
  int objective;              /* CHNS_PC_OBJ_*                               */
} chns_pc_batch;
int chns_pc_train_step(chns_ctx* ctx, const chns_pc_batch* batch, float lr, float* loss, void* stream);

/* ------------------------------------------------------------ profiling */

/* Per-kernel timers (paper Sec. 6 reports per-solver time breakdowns; these
 * are the device analogue).  When enabled, the context records HIP events
 * on the caller's stream around each tagged launch group: "pp_brick_fp64",
 * "pp_brick_fp32", "mass_brick_fp64", "massrho_brick_fp64", "combine", ...
 * chns_profile_read synchronises the pending events and returns the summed
 * milliseconds and number of launch groups for `tag` since the last reset. */
int chns_profile_enable(chns_ctx* ctx, int enable);
int chns_profile_read(chns_ctx* ctx, const char* tag, double* ms, int64_t* launches);
int chns_profile_reset(chns_ctx* ctx);

/* Last error message of the calling thread ("" if none). */
const char* chns_last_error(void);
/* Library version string. */
const char* chns_version(void);

#ifdef __cplusplus
}
#endif
#endif /* CHNS_H */
