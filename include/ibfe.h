/*
 * ibfe.h - C ABI of the MI355X (gfx950) IPCS + BCE-IB finite-element time step.
 *
 * The library advances the incompressible Navier-Stokes equations with an
 * immersed boundary (Bourantas et al., "Immersed boundary finite element method
 * for blood flow simulation", Section 2): each step is the incremental pressure
 * correction scheme of Section 2.2 (tentative velocity, pressure increment,
 * velocity/pressure correction) combined with the boundary-condition-enforced IB
 * correction of Section 2.3 in the order of Section 2.4.  The discretisation is
 * trilinear (Q1) on a uniform Cartesian grid reduced to the vessel by a node
 * mask (domain reduction, Section 4).
 *
 * Conventions
 *  - Grid: nx*ny*nz cells of side h, nodes (i,j,k) with 0<=i<=nx etc., node id
 *    n = i + (nx+1)*(j + (ny+1)*k) (x fastest), N = (nx+1)(ny+1)(nz+1).
 *  - Kept cells: cells with at least one corner of mask 1.  P = corners of kept
 *    cells: velocity and pressure live on P, in ascending node id ("canonical
 *    order"); every array exchanged through this ABI uses that order.
 *  - Velocity arrays are structure-of-arrays: u[d*n + q] is component d of the
 *    q-th node of P.  All floating point data crossing the ABI is FP64.
 *  - Return codes: 0 on success, a negative IBFE_E* code on failure;
 *    ibfe_last_error() returns a thread-local message for the last failure.
 *  - Host arrays passed in are copied before the call returns; the caller keeps
 *    ownership.  Device memory is obtained from the caller's allocator if one is
 *    given (else hipMalloc) and belongs to the context until ibfe_destroy.  The
 *    HIP stream is borrowed: every kernel of a context runs on it.
 *  - A context is not thread-safe; different contexts may be used concurrently
 *    from different threads on different streams.
 */
#ifndef IBFE_H
#define IBFE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define IBFE_OK 0
#define IBFE_EINVAL (-1)     /* bad shape, value or call order                      */
#define IBFE_ENOMEM (-2)     /* device or host allocation failed                     */
#define IBFE_EHIP (-3)       /* HIP runtime error (no device, launch failure)        */
#define IBFE_ENOCONV (-4)    /* a Krylov solve hit its iteration cap                 */
#define IBFE_ENONFINITE (-5) /* NaN/Inf in a residual                                */
#define IBFE_ESINGULAR (-6)  /* Lagrangian point without free support / breakdown    */

/* Boundary tags per node (only meaningful on box-face nodes). */
#define IBFE_TAG_NONE 0
#define IBFE_TAG_WALL 1
#define IBFE_TAG_INLET 2
#define IBFE_TAG_OUTLET 3

/* Node flag bits returned by ibfe_plan_node_flags. */
#define IBFE_FLAG_P 1u      /* corner of a kept cell                            */
#define IBFE_FLAG_F 2u      /* free velocity node                               */
#define IBFE_FLAG_DU 4u     /* velocity Dirichlet node                          */
#define IBFE_FLAG_PDIR 8u   /* pressure Dirichlet (outlet) node                 */
#define IBFE_FLAG_HANG 32u  /* hanging lattice node of a refined grid (not in P) */

/*
 * Grid and domain reduction (Section 2.3: uniform Cartesian Eulerian nodes of
 * spacing h; Section 4: elements outside the vessel removed).
 *   node_mask : N bytes, 1 = inside the vessel, 0 = outside (required)
 *   bc_tag    : N bytes of IBFE_TAG_*, or NULL for the defaults: z = 0 face
 *               inlet, z = nz face outlet, the x and y faces wall, wall winning
 *               on shared edges/corners.
 *   refine_cell: nx*ny*nz bytes (cell c = i + nx*(j + ny*k)), 1 = split the
 *               cell 2:1, or NULL for a uniform grid.
 * Velocity Dirichlet nodes D_u: nodes of P with mask 0 (value 0), wall-tagged
 * nodes of P (value 0), inlet-tagged nodes of P (inlet table value, else 0).
 * Free velocity nodes F = P \ D_u.  Pressure Dirichlet: outlet-tagged nodes of
 * P (pressure increment 0).  A connected part of the kept region without an
 * outlet node has its pressure increment normalised to zero nodal mean.
 *
 * Local 2:1 refinement (the paper refines its mesh near the immersed boundary,
 * Section 4).  With refine_cell, nx, ny, nz and h describe the base grid and
 * every node array (node_mask, bc_tag, inlet node ids, the canonical ids
 * returned by the library) lives on the fine lattice of (2nx+1)(2ny+1)(2nz+1)
 * nodes of spacing h/2, id n = i + (2nx+1)*(j + (2ny+1)*k).  Elements: the
 * 2x2x2 children (side h/2) of flagged cells and the unflagged cells (side h),
 * each kept when one of its 8 corners has mask 1.  A lattice node that is a
 * corner of a kept child and lies strictly inside an edge or a face of a kept
 * unflagged cell is hanging: its value is the mean of the 2 edge end points or
 * the 4 face corners, and every operator is C^T A C with that constraint C.
 * P = corners of kept elements minus hanging nodes; the sets above follow on
 * the lattice.  The IB kernel uses the lattice spacing h/2, and every support
 * node of every Lagrangian point must lie in the closure of a flagged cell and
 * not be hanging (else IBFE_EINVAL).  Inlet table entries at lattice nodes
 * outside P (interior points of unflagged cells, hanging nodes) are skipped.
 */
typedef struct ibfe_grid {
  int32_t nx, ny, nz;
  double h;
  double origin[3];
  const uint8_t* node_mask;
  const uint8_t* bc_tag;
  const uint8_t* refine_cell;
} ibfe_grid;

/*
 * Lagrangian wall points (Section 2.3, Eqs. 17-24): X is M x 3 (row major),
 * dS the uniform surface element of each point (Section 2.5), U_B the
 * prescribed wall velocity, M x 3, or NULL for a wall at rest.  The IB
 * correction solves G Lambda = U_B - I u* with G = I_F I_F^T, where
 * I_ij = prod_d delta4((x_j,d - X_i,d)/h) over the 4x4x4 support starting at
 * floor((X_i - origin)/h) - 1 (Eq. 17 times h^3, kernel of Eq. 18); support
 * nodes outside the box are dropped.  Every point needs
 * sum_{j in F} I_ij^2 >= 1e-12, else IBFE_ESINGULAR.  M may be 0.
 */
typedef struct ibfe_ib {
  int64_t M;
  const double* X;
  double dS;
  const double* U_B;
} ibfe_ib;

/*
 * Physical and numerical parameters.
 *   rho, mu, dt : density, dynamic viscosity, time step (all > 0)
 *   precision   : 0 = FP64 throughout; 1 = FP32 inner Krylov solves inside FP64
 *                 iterative refinement (FP64 outer residuals, dots, IB solve)
 *   rtol        : relative residual target of the velocity and pressure solves
 *                 (<= 0 selects 1e-13 in FP64 mode, 1e-8 in mixed mode)
 *   max_iters   : iteration cap per Krylov solve (<= 0 selects 20000)
 *   precond     : preconditioner of the pressure increment CG (Jacobi for the
 *                 other solves): 0 = Jacobi; 1 = Chebyshev-Jacobi polynomial of
 *                 degree 16 on [lambda_max/4, lambda_max] of D^-1 K with the bound
 *                 lambda_max = 2; 2 = geometric multigrid V(1,1) cycle with
 *                 Chebyshev-Jacobi smoothing and a dense coarsest solve
 *   advection   : 0 = semi-implicit u^n . grad u* (BiCGStab on the advection-
 *                 diffusion operator); 1 = explicit u^n . grad u^n (the convection
 *                 of Eq. 13 at the old velocity on the right-hand side; CG on the
 *                 symmetric (rho/dt) M + mu K)
 *   ib_rtol     : relative residual target of the IB force solve (<= 0: 1e-13 with
 *                 precision 0, 1e-10 with precision 1)
 *   viscous     : viscous form of the momentum equation (Section 2.1): 0 = the
 *                 component-wise mu (grad u, grad v); 1 = the strain-rate form
 *                 2 mu (eps(u), eps(v)), eps(u) = (grad u + grad u^T)/2, which
 *                 couples the three components of the tentative-velocity system
 *                 (uniform and refined grids, either advection)
 *   advdiff     : how the semi-implicit tentative-velocity operator
 *                 (rho/dt) M + rho C(u^n) + mu K of Eq. 9 is applied: 0 = matrix-free
 *                 (each row formed from the cell bits and u^n at its 27 neighbours
 *                 on every apply; nothing stored); 1 = a stencil of 27 coefficients
 *                 per node (54 on a refined lattice) assembled once per step and
 *                 streamed by every apply.  Both give the same operator up to
 *                 rounding.  The explicit advection option always assembles the
 *                 stencil of rho C(u^n) for its one product per step.
 *   mass_precond : preconditioner of the Chebyshev iteration of the consistent-
 *                 mass correction M_FF delta = (G Phi)_F (Sections 2.2 and 2.4):
 *                 0 = Jacobi, on the proven interval [1/8, 27/8] of D^-1 M (on a
 *                 refined lattice with the lumped constrained diagonal); 1 = the
 *                 tensor-product approximate inverse D^-1/2 T D^-1/2 (T the
 *                 product of the stencils (-1/4, 1, -1/4) along the axes, among
 *                 the fine rows at lattice spacing and among the rows with coarse
 *                 cells at twice that spacing), whose spectrum on the interior
 *                 is [27/64, 1]; the iteration takes [0.4, 1.6] and converges for
 *                 every eigenvalue in (0, 2).  Three to four times fewer steps of
 *                 two passes each.  The batcher of ibfe_batcher_create joins
 *                 only mass_precond = 0 solves.
 */
typedef struct ibfe_params {
  double rho, mu, dt;
  int32_t precision;
  double rtol;
  int32_t max_iters;
  int32_t precond;
  int32_t advection;
  double ib_rtol;
  int32_t viscous;
  int32_t advdiff;
  int32_t mass_precond;
} ibfe_params;

/*
 * Inlet velocity table (the paper prescribes a parabolic inlet profile in the
 * angle-tube test of Section 3.2 and a pulsatile inlet waveform with a parabolic
 * profile in the coronary example of Section 4.1; a Fourier series in time with a
 * spatial shape per harmonic covers both).  The prescribed velocity at table node
 * q and time t is
 *   u_in = W_0 + sum_{k=1..K} [ Re W_k cos(k omega t) - Im W_k sin(k omega t) ]
 * (the real part of sum_k W_k e^{i k omega t}).  shape holds (2K+1) blocks of
 * n x 3 doubles: W_0, Re W_1, Im W_1, ..., Re W_K, Im W_K (each block row major
 * n x 3).  Every listed node must be an inlet-tagged node of P with mask 1.
 */
typedef struct ibfe_inlet {
  int32_t K;
  double omega;
  int64_t n;
  const int64_t* node_ids;
  const double* shape;
} ibfe_inlet;

/* Device allocator used for every device buffer of a context.  alloc returns
 * NULL on failure; stream is the context's stream. */
typedef struct ibfe_alloc {
  void* (*alloc)(size_t bytes, void* stream, void* user);
  void (*free)(void* ptr, void* user);
  void* user;
} ibfe_alloc;

/* Statistics of the last completed step. */
typedef struct ibfe_stats {
  int64_t steps;          /* completed steps since the last ibfe_set_state      */
  double t;               /* current time                                       */
  int32_t s1_iters;       /* tentative velocity solve (BiCGStab iterations)     */
  int32_t ib_iters;       /* IB force solve (CG iterations)                     */
  int32_t s3_iters;       /* pressure increment solve (CG iterations)           */
  int32_t s4_iters;       /* velocity correction solve (Chebyshev steps)        */
  int32_t s1_outer, s3_outer, s4_outer; /* refinement sweeps (mixed mode)       */
  double s1_res, ib_res, s3_res, s4_res; /* final relative residuals            */
  double poisson_apply_ms;   /* summed duration of the pressure stiffness apply  */
  int64_t poisson_applies;   /* and its dispatches (kernel timing on, see below)  */
  double mass_apply_ms;      /* summed duration of the mass Chebyshev steps of   */
  int64_t mass_applies;      /* the velocity correction, and their number        */
  int32_t s1_restarts;       /* BiCGStab restarts after a breakdown (r^.v = 0 or  */
  int32_t reserved_;         /* t.t = 0 before convergence), at most 3 per solve */
} ibfe_stats;

typedef struct ibfe_plan ibfe_plan;
typedef struct ibfe_ctx ibfe_ctx;

/* ---- host-only set-up (no GPU needed) ---------------------------------- */

/* Validate the inputs and derive kept cells, P, F, D_u, pressure Dirichlet
 * nodes, the canonical order and the IB stencils on the host. */
int ibfe_plan_create(const ibfe_grid* grid, const ibfe_ib* ib, const ibfe_params* params,
                     const ibfe_inlet* inlet, ibfe_plan** out);
/* Sizes: |P|, |F|, |P minus outlet|, kept cells, outlet-less components. */
int ibfe_plan_sizes(const ibfe_plan* plan, int64_t* n_p, int64_t* n_free, int64_t* n_pfree,
                    int64_t* n_kept_cells, int64_t* n_floating);
/* Node ids of P in canonical (ascending) order: n_p int64 values. */
int ibfe_plan_node_ids(const ibfe_plan* plan, int64_t* ids);
/* IBFE_FLAG_* bits for every one of the N grid nodes. */
int ibfe_plan_node_flags(const ibfe_plan* plan, uint8_t* flags);
void ibfe_plan_destroy(ibfe_plan* plan);

/* ---- device context ----------------------------------------------------- */

/* Create a context on the current HIP device.  alloc may be NULL (hipMalloc);
 * hip_stream is a hipStream_t (NULL = the null stream).  The initial state is
 * u = 0, p = 0, t = 0. */
int ibfe_create(const ibfe_grid* grid, const ibfe_ib* ib, const ibfe_params* params,
                const ibfe_inlet* inlet, const ibfe_alloc* alloc, void* hip_stream,
                ibfe_ctx** out);
/* Number of velocity nodes and pressure nodes (both |P|). */
int ibfe_num_nodes(const ibfe_ctx* ctx, int64_t* n_u, int64_t* n_p);
/* Canonical node ids of the velocity and pressure unknowns (either may be NULL). */
int ibfe_get_node_ids(const ibfe_ctx* ctx, int64_t* vel_ids, int64_t* p_ids);
/* Set u (3 x n_u SoA), p (n_p) and t.  on_device != 0: pointers are device
 * memory readable on the context's stream; else host memory. */
int ibfe_set_state(ibfe_ctx* ctx, const double* u, const double* p, double t, int on_device);
/* Advance nsteps steps (Section 2.4).  On failure the state of the last
 * completed step is kept. */
int ibfe_step(ibfe_ctx* ctx, int nsteps);
/* Move the Lagrangian points (Section 2.3 defines I, I_F and the force system
 * G = I_F I_F^T for the current positions): X (M x 3, row major) are the
 * positions and U_B (M x 3, NULL = 0) the prescribed velocities that the next
 * steps enforce; M is the count given at ibfe_create.  The stencils of Eq. 17,
 * the spreading lists, G and its block-Jacobi preconditioner are rebuilt on the
 * device (deterministic: the same positions give the same G on every call).
 * on_device != 0: X and U_B are device memory (not validated); else host memory
 * (must be finite, IBFE_EINVAL).  On a refined lattice every support node must
 * stay in the closure of a flagged cell and not be hanging, as at ibfe_create
 * (else IBFE_EINVAL).  IBFE_ESINGULAR if a point's support holds no free node; IBFE_EINVAL if
 * the points are so dense that a row of G collects more than 1024 support
 * products.  After an error the context refuses to step until a call succeeds.
 * The first call allocates the rebuild buffers (about 1.6 KB per point) and
 * drops captured graphs; every call synchronises the stream twice. */
int ibfe_set_points(ibfe_ctx* ctx, const double* X, const double* U_B, int on_device);
/* ibfe_set_points for callers that cannot allocate device memory (code under HIP
 * graph capture, allocation-free time loops): the same rebuild with the same
 * results, its scratch (positions, sorted support pairs, scan and sort work,
 * counters: about 1.6 KB per point) taken from a 32 MiB array that the library
 * holds per GPU for the life of the process, instead of buffers allocated on the
 * first call.  The context's spreading lists and G are preallocated at
 * ibfe_create, so nothing is allocated here.  IBFE_EINVAL if the points need more
 * scratch than the array holds (M > ibfe_set_points_noalloc_max_points()).  Every
 * call on one GPU uses the same array: calls that overlap on a GPU (other
 * threads, other streams) race and must be serialised by the caller.  The
 * stream is synchronised twice, as in ibfe_set_points. */
int ibfe_set_points_noalloc(ibfe_ctx* ctx, const double* X, const double* U_B, int on_device);
/* Largest number of Lagrangian points ibfe_set_points_noalloc accepts. */
int64_t ibfe_set_points_noalloc_max_points(void);
/* Advance until the flow is steady (Section 3.1): after every step, the
 * step-to-step normalised root-mean-square difference of each velocity
 * component d,
 *   L_d = sqrt(sum_i (u_d,i^{n+1} - u_d,i^n)^2 / N^2) / (max_i u_d,i^n - min_i u_d,i^n),
 * over the N = n_u nodes of P (a component with max = min: 0 if it did not
 * change, +inf if it did), is computed on the device; stop as soon as all three
 * are below tol, or after max_steps steps.  steps (host) receives the number of
 * steps taken, nrmse (host, 3 values) the last step's L_d (all +inf when no step
 * was taken): the steady state was reached iff all three are below tol.  A
 * failed step returns its error with the last completed state kept.
 * Synchronises the stream once per step. */
int ibfe_run_steady(ibfe_ctx* ctx, double tol, int64_t max_steps, int64_t* steps, double* nrmse);
/* Read u, p (either may be NULL) and t; synchronises the stream for host output. */
int ibfe_get_state(ibfe_ctx* ctx, double* u, double* p, double* t, int on_device);

/* Checkpoint and restart of the time stepping (Section 2.4 advances (u^n, p^n) to
 * (u^{n+1}, p^{n+1}); the library also carries, from one step to the next, the
 * initial guesses of its iterative solves: the IB force Lambda of Eq. 23, the
 * pressure increment Phi of Eq. 12 and the mass correction of the velocity
 * update).  A checkpoint holds u, p, t, the step count and those three guesses, so
 * that k steps, save, load into a context created from the same inputs, and
 * N - k more steps give bitwise the state of N uninterrupted steps (ibfe_set_state
 * instead starts the solves cold: the same state within the solver tolerances).
 * Layout: a 48-byte header (magic "IBFECKP1", n_p, M, t, steps, flags), then FP64
 * arrays in canonical order: u (3 x n_u), p (n_p), Phi (n_p), the mass correction
 * (3 x n_u), Lambda (3 x M, component planes).  buf is host memory of at least
 * ibfe_checkpoint_size bytes; the caller owns it.  Moved Lagrangian points are
 * not part of the checkpoint: call ibfe_set_points again after a load.
 * ibfe_checkpoint_load refuses (IBFE_EINVAL) a buffer whose header does not match
 * the context's sizes.  Both calls synchronise the stream. */
int ibfe_checkpoint_size(const ibfe_ctx* ctx, size_t* bytes);
int ibfe_checkpoint_save(ibfe_ctx* ctx, void* buf, size_t bytes);
int ibfe_checkpoint_load(ibfe_ctx* ctx, const void* buf, size_t bytes);

/* Testing aid for the failure paths: make the next tentative-velocity BiCGStab
 * solve of this context report a breakdown once its iteration count reaches
 * `iteration` (> 0; 0 cancels), as if r^.v or t.t had vanished.  The solver then
 * restarts from its current iterate (ibfe_stats.s1_restarts counts it).  No
 * effect on the CG paths (advection = 1). */
int ibfe_inject_breakdown(ibfe_ctx* ctx, int iteration);
int ibfe_get_stats(const ibfe_ctx* ctx, ibfe_stats* stats);
/* Enable (1) or disable (0) per-dispatch kernel timing: while on, every kernel
 * dispatch of the context records its own start and end events, and the
 * durations are summed per kernel name at the end of every step (dispatches of
 * Krylov iterations past convergence, which return at once, are not counted).
 * Graph replay is off meanwhile (the kernels are dispatched one by one, with the
 * same results).  Both calls reset the sums, and the two summary fields of
 * ibfe_stats: poisson_apply_ms / poisson_applies (the pressure stiffness apply
 * k_cg_q_zb<*, 1>) and mass_apply_ms / mass_applies (the mass Chebyshev step of
 * the velocity correction: k_zb_cheb<*, false, 3, *> with mass_precond = 0, the
 * update pass k_tm_cheb<*, 3, *, *> with mass_precond = 1). */
int ibfe_set_kernel_timing(ibfe_ctx* ctx, int enable);

/* Summed durations per kernel since timing was enabled, longest total first:
 * up to cap entries are written to out (host memory), *n receives the number
 * of kernels.  name is the kernel's instantiation as the compiler spells it
 * (for example "k_zb_cheb<float, false, 3>").  Synchronises the stream. */
typedef struct ibfe_kernel_time {
  char name[120];
  double total_ms;
  int64_t launches;
} ibfe_kernel_time;
int ibfe_get_kernel_times(ibfe_ctx* ctx, ibfe_kernel_time* out, int32_t cap, int32_t* n);
/* Time only the dispatches of the named kernel (a name as ibfe_get_kernel_times
 * spells it), or every kernel (NULL or "").  Events on every dispatch slow the
 * step (about 5 us per dispatch); one kernel's events do not measurably. */
int ibfe_set_kernel_timing_filter(ibfe_ctx* ctx, const char* kernel);

/* Replay the fixed kernel sequences of the solves (iteration batches between
 * convergence checks, Chebyshev sequences) through HIP graphs captured on their
 * first use (1, the default) or launch every kernel directly (0).  Graphs are
 * only used on a non-null stream and not while kernel timing is enabled; the
 * results are bitwise the same either way.  Switching frees the graphs. */
int ibfe_set_graphs(ibfe_ctx* ctx, int enable);

/* Wall shear stress at the Lagrangian points for the current velocity (the
 * paper's clinical output, defined in Section 2.6, evaluated at the immersed wall points):
 * the nodal velocity gradient by the lumped L2 projection of the Q1 gradient,
 * g_de = (G_e u_d) / m with m the row sum of the mass matrix, its symmetric part
 * eps interpolated to each point with the kernel of Eq. 18 (the weights of the
 * IB interpolation), and the tangential part tau = t - (t . n) n of the traction
 * t = 2 mu eps n.
 *   normals : M x 3 row major, wall normal of each point (scaled to unit length;
 *             host memory, or device memory with on_device = 1)
 *   tau     : M x 3 row major output, same memory kind
 * On a refined lattice the gradients are the composite ones (hanging values
 * constrained to their parents) and m the row sums of the constrained mass.
 * IBFE_EINVAL without points.  Uses the context's work space and synchronizes
 * its stream. */
int ibfe_wall_shear(ibfe_ctx* ctx, const double* normals, double* tau, int on_device);

/* Intermediate fields of the last step, canonical order:
 *   IBFE_FIELD_USTAR (3 x n_u)  tentative velocity after the first sub-step
 *   IBFE_FIELD_UIB   (3 x n_u)  velocity after the IB correction
 *   IBFE_FIELD_PHI   (n_p)      pressure increment */
#define IBFE_FIELD_USTAR 0
#define IBFE_FIELD_UIB 1
#define IBFE_FIELD_PHI 2
int ibfe_get_field(ibfe_ctx* ctx, int which, double* out, int on_device);

/* Apply one discrete operator of the step (for verification), canonical order,
 * rows on all of P, columns on all of P:
 *   IBFE_OP_MASS    y = M x            x: n_p,      y: n_p
 *   IBFE_OP_STIFF   y = K x            x: n_p,      y: n_p
 *   IBFE_OP_GRAD    y_d = G_d x        x: n_p,      y: 3 x n_u
 *   IBFE_OP_DIV     y = sum_d G_d x_d  x: 3 x n_u,  y: n_p
 *   IBFE_OP_ADVDIFF y_d = A x_d with A = (rho/dt) M + rho C(u) + mu K and u the
 *                   current state velocity      x: 3 x n_u, y: 3 x n_u
 *                   (viscous = 1: plus mu sum_c X_dc x_c, the strain-rate cross
 *                   blocks X_dc = int d_c N_i d_d N_j)
 *   IBFE_OP_INTERP  y = I x            x: 3 x n_u,  y: M x 3 (row major)
 *   IBFE_OP_SPREAD  y = I_F^T x        x: M x 3,    y: 3 x n_u
 * precision 0 runs the FP64 kernels, 1 the FP32 kernels (MASS, STIFF, ADVDIFF;
 * others are FP64 only).  Host or device pointers as for ibfe_set_state. */
#define IBFE_OP_MASS 0
#define IBFE_OP_STIFF 1
#define IBFE_OP_GRAD 2
#define IBFE_OP_DIV 3
#define IBFE_OP_ADVDIFF 4
#define IBFE_OP_INTERP 5
#define IBFE_OP_SPREAD 6
int ibfe_apply(ibfe_ctx* ctx, int op, int precision, const double* x, double* y, int on_device);

void ibfe_destroy(ibfe_ctx* ctx);
const char* ibfe_last_error(void);

/* ---- batched kernels across contexts ------------------------------------- */

/*
 * A batcher joins the consistent-mass Chebyshev sequences of several contexts
 * into single launches (the velocity correction, the last step of the scheme
 * of Section 2.2 and of the algorithm of Section 2.4, is taken with the
 * consistent mass and solved by Chebyshev iteration inside the FP64
 * refinement): each Chebyshev step is one kernel over the column items of every
 * context that reached that stage, instead of one kernel per context.  It
 * applies to mixed-precision contexts on uniform grids (others keep their own
 * launches).  A context whose thread reaches the stage waits up to
 * window_us microseconds for the other attached contexts to join (not at all
 * when it is the only one attached); the batch runs on the batcher's own
 * stream, ordered after each member's earlier work by events, and each member's
 * stream waits for the batch before its next kernel.  Every node's arithmetic
 * is that of the context's own launch, so results are bitwise identical with
 * and without a batcher.  Contexts that step from different host threads share
 * it; a context must be detached (or destroyed) before its batcher is.
 */
typedef struct ibfe_batcher ibfe_batcher;
/* Create a batcher on the current HIP device. */
int ibfe_batcher_create(double window_us, ibfe_batcher** out);
/* Attach ctx to batcher b (NULL detaches); IBFE_EINVAL for another device. */
int ibfe_attach_batcher(ibfe_ctx* ctx, ibfe_batcher* b);
/* Batches launched, member sequences they carried, and the widest batch. */
int ibfe_batcher_stats(ibfe_batcher* b, int64_t* batches, int64_t* members, int32_t* widest);
/* Release a batcher with no attached context (IBFE_EINVAL otherwise). */
int ibfe_batcher_destroy(ibfe_batcher* b);

/* ---- serving: continuous batching of independent flow solves ------------- */

/* One flow solve: the inputs of ibfe_create plus the number of steps, starting
 * from rest (u = 0, p = 0) at time t0.  All arrays are copied by submit. */
typedef struct ibfe_request {
  const ibfe_grid* grid;
  const ibfe_ib* ib;
  const ibfe_params* params;
  const ibfe_inlet* inlet;
  int32_t nsteps;
  double t0;
} ibfe_request;

#define IBFE_REQ_QUEUED 0
#define IBFE_REQ_RUNNING 1
#define IBFE_REQ_DONE 2
#define IBFE_REQ_FAILED 3

/* Progress and timing of a request (times in seconds since server creation). */
typedef struct ibfe_result {
  int32_t status;       /* IBFE_REQ_*                                        */
  int32_t error;        /* IBFE_E* code when FAILED                          */
  int64_t n_u, n_p;     /* sizes of the fetched arrays (valid when DONE)     */
  size_t footprint;     /* device bytes reserved for the request            */
  double t_submit, t_admit, t_done;
  ibfe_stats stats;     /* statistics of the last step                       */
} ibfe_result;

typedef struct ibfe_server ibfe_server;

/* Device bytes a request reserves (estimate from the grid size, the number
 * of Lagrangian points, precision and preconditioner; an upper bound of what
 * its context allocates). */
int ibfe_request_footprint(const ibfe_request* req, size_t* bytes);

/* Create a server on the current HIP device with max_slots worker slots (each
 * slot runs one request at a time on its own HIP stream; slots run
 * concurrently, so admitted requests overlap on the GPU).  budget_bytes caps
 * the summed footprint of running requests (0 = 90 % of the free device
 * memory).  Requests are admitted first-in first-out as slots and memory free
 * up; a request larger than the budget fails with IBFE_ENOMEM at submit. */
int ibfe_server_create(size_t budget_bytes, int32_t max_slots, ibfe_server** out);
/* Queue a request; returns at once with its id. */
int ibfe_server_submit(ibfe_server* srv, const ibfe_request* req, int64_t* id);
/* Current status of a request (non-blocking). */
int ibfe_server_poll(ibfe_server* srv, int64_t id, ibfe_result* out);
/* Block until the request is DONE or FAILED, or timeout_s elapses (< 0: no limit). */
int ibfe_server_wait(ibfe_server* srv, int64_t id, double timeout_s, ibfe_result* out);
/* Copy the final state of a DONE request (canonical order, host memory; any
 * pointer may be NULL) and release it; node_ids receives n_u ids. */
int ibfe_server_fetch(ibfe_server* srv, int64_t id, double* u, double* p, int64_t* node_ids);
/* Largest number of requests that ran at the same time so far. */
int ibfe_server_peak_concurrency(const ibfe_server* srv, int32_t* peak);
/* Batch the mass-correction kernels of the running requests (a batcher with
 * the given window shared by every request admitted after the call; see
 * ibfe_batcher_create); call before submitting.  stats as ibfe_batcher_stats
 * (zeros when batching is off). */
int ibfe_server_set_batching(ibfe_server* srv, double window_us);
int ibfe_server_batch_stats(ibfe_server* srv, int64_t* batches, int64_t* members, int32_t* widest);
/* Finish running requests, fail the queued ones, release everything. */
void ibfe_server_destroy(ibfe_server* srv);

#ifdef __cplusplus
}
#endif
#endif /* IBFE_H */
