/*
 * hwe.h -- C ABI of the MI355X (gfx950) explicit step of the compact
 * ADER-HWENO finite-volume scheme on triangular meshes
 * (Luo, Zhao, Qiu, Chen: "A compact simple HWENO scheme with ADER time
 * discretization for hyperbolic conservation laws II: triangular meshes").
 *
 * The scheme advances, for every triangle K, the cell average of the solution
 * W and the cell averages of W_x and W_y (Sec. 2.2, eq. (aver)) by one
 * explicit step (eq. (flx) for the averages of W; eqs. (derave2d1)-(derave2d2)
 * for the derivative averages).  Only plain pointers and sizes cross this
 * boundary; no C++ or torch types.
 *
 * Conventions shared by every entry point
 *  - Every function returns hwe_status (HWE_OK = 0).  On failure a message is
 *    available from hwe_last_error() (thread-local) and no work is launched.
 *  - Device pointers are HIP device memory on the mesh's device; "stream" is a
 *    hipStream_t passed as void* (NULL = the default stream).  Launches are
 *    asynchronous on that stream; the library never synchronises the device
 *    inside hwe_step / hwe_step_adjoint.  Device faults surface at the caller's
 *    next synchronisation.
 *  - Cell order: the library renumbers cells along a Morton curve of their
 *    centroids.  All state buffers are in this internal order;
 *    hwe_mesh_cell_perm() gives the map to the caller's triangle order.
 *  - State layout (structure of arrays, component-major):
 *      wbar : double [m][N]          cell averages of W         (eq. (aver))
 *      grad : [2][m][N]              averages of W_x, then W_y  (eq. (aver))
 *             double for HWE_FP64, float for HWE_MIXED
 *    m = 1 (advection, Burgers) or 4 (Euler: rho, rho u, rho v, E).
 *  - A mesh handle owns device scratch, and two calls that use the same
 *    scratch must not overlap in time (on one stream they serialise by
 *    themselves).  The scratch sets: hwe_step and hwe_step_keep use the edge
 *    fluxes (hwe_step also the reconstruction); hwe_step_adjoint and
 *    hwe_step_adjoint_kept use the adjoint records (hwe_step_adjoint also the
 *    reconstruction); hwe_max_dt and hwe_check_state one reduction buffer
 *    each.  So hwe_step_keep on one stream may overlap hwe_step_adjoint_kept
 *    on another (a checkpointed reverse sweep recomputes the next segment
 *    beside the current one's adjoints), while two steps, or two adjoints,
 *    may not.  The profiling events (hwe_profile_begin) assume one stream.
 *  - On a mesh with reflective walls or prescribed boundary states the two
 *    adjoint calls fork part of their work onto a stream the handle owns
 *    (default priority, created with the handle) and join it back into the
 *    caller's stream by events before their next launch there: the work
 *    starts after what precedes the call on the caller's stream and is
 *    complete before what follows it, and a graph captured from that stream
 *    holds the forked branch.  That stream belongs to the adjoint's scratch
 *    set above.
 *  - Memory given by the caller is never freed or reallocated by the library.
 */
#ifndef HWE_H
#define HWE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hwe_mesh_s* hwe_mesh; /* opaque, library-owned */

typedef enum {
  HWE_OK = 0,
  HWE_EINVAL = -1,     /* bad argument (null, aliasing, dt <= 0 or not finite, size) */
  HWE_EMESH = -2,      /* degenerate / non-manifold / unmatched periodic mesh */
  HWE_ESINGULAR = -3,  /* rank-deficient reconstruction least-squares system */
  HWE_ENOMEM = -4,     /* host or device allocation failed */
  HWE_EHIP = -5,       /* a HIP runtime call or kernel launch failed */
  HWE_ENODEV = -6      /* operation needs a device but the handle is host-only */
} hwe_status;

typedef enum { HWE_ADVECTION = 0, HWE_BURGERS = 1, HWE_EULER = 2 } hwe_equation;
typedef enum { HWE_BC_PERIODIC = 0, HWE_BC_TRANSMISSIVE = 1 } hwe_bc;
typedef enum { HWE_FP64 = 0, HWE_MIXED = 1 } hwe_precision;

/* Boundary kinds of a region (Sec. 4's boundary conditions on generated
 * meshes).  HWE_BND_TRANSMISSIVE: outflow, the ghost cell is the mirror image
 * of the cell with its state, the exterior value is the interior one.
 * HWE_BND_WALL (Euler): reflective, as for opts.walls.  HWE_BND_STATE_A / _B:
 * inflow, a prescribed state: the ghost cell holds it with zero derivative
 * averages and it is the exterior value at every time node.
 * HWE_BND_MOVING: state A where the face midpoint has
 * x < shock_x0 + shock_speed * t, else state B, with t the middle of the step
 * (the exact position of a shock meeting the boundary, as on the top of the
 * double Mach reflection problems). */
typedef enum {
  HWE_BND_TRANSMISSIVE = 0,
  HWE_BND_WALL = 1,
  HWE_BND_STATE_A = 2,
  HWE_BND_STATE_B = 3,
  HWE_BND_MOVING = 4
} hwe_bnd_kind;

#define HWE_MAX_REGIONS 8

typedef struct {
  int32_t kind;   /* hwe_bnd_kind */
  int32_t pad;
  double box[4];  /* x0, x1, y0, y1: boundary faces whose midpoint lies in this
                     closed rectangle (a side: x0 == x1 or y0 == y1) */
} hwe_region;

typedef struct {
  int32_t eq;             /* hwe_equation; linear advection u_t + a.grad u = 0,
                             Burgers (Example 4.1), Euler gamma-law gas (eq. (2d)) */
  int32_t bc;             /* hwe_bc: periodic (box is the period) or transmissive */
  int32_t prec;           /* hwe_precision.  HWE_MIXED: FP32 tables, derivative
                             averages, reconstruction coefficients, Lax-Wendroff and
                             fluxes; FP64 cell averages of W, their accumulation,
                             smoothness-indicator sums and nonlinear weights */
  int32_t linear_weights; /* 1: omega = gamma (Step 3 weights only); 0: the
                             nonlinear weights of Step 5, eq. (nonlinearweight) */
  double box[4];          /* x0, x1, y0, y1 of the domain */
  double adv[2];          /* advection velocity (HWE_ADVECTION) */
  double gas_gamma;       /* ratio of specific heats (HWE_EULER), e.g. 1.4 */
  double lin_w[4];        /* linear weights gamma_1..gamma_4 (Step 3): 0.94, 0.02 x3 */
  double eps;             /* epsilon of eq. (nonlinearweight): 1e-8 */
  int32_t device;         /* HIP device ordinal; -1 = host precompute only (no
                             device memory; hwe_step etc. return HWE_ENODEV) */
  int32_t positivity;     /* 1 (Euler only): positivity-preserving scaling of the
                             reconstruction about the cell average (the scale
                             limiter cited in Sec. 3): density, then pressure, kept
                             >= min(1e-13, average density, average pressure) at
                             the cell's six edge Gauss points.  0: off */
  int32_t time_rule;      /* quadrature of the time integral in eq. (flux):
                             0 = 3-point Gauss-Lobatto, nodes {0, 1/2, 1} dt,
                             weights {1, 4, 1}/6 (default); 1 = 2-point
                             Gauss-Legendre, nodes (1/2 -+ sqrt(3)/6) dt, weights
                             1/2.  The interface value of eq. (timeflux) is the
                             Taylor polynomial at dt with either rule */
  double deriv_weight;    /* weight w > 0 of the two derivative rows in the
                             Step-2 least squares of Sec. 2.2 (the linear
                             candidates); 1 = the rows as printed (default) */
  int32_t walls;          /* HWE_EULER with HWE_BC_TRANSMISSIVE only: bit s set
                             (s = 0: x = x0, 1: x = x1, 2: y = y0, 3: y = y1)
                             makes the boundary faces lying on that side of the
                             box reflective walls: the ghost cell is the mirror
                             image of the cell with its momentum reflected, and
                             the exterior value at a wall Gauss point is the
                             interior value with its momentum reflected.  Other
                             boundary faces stay transmissive.  0 = no walls
                             (default) */
  int32_t n_regions;      /* HWE_BC_TRANSMISSIVE only: 0..HWE_MAX_REGIONS.  Each
                             boundary face takes the kind of the first region
                             that holds its midpoint (within 1e-9 of the box
                             size); faces in no region follow `walls`.  Walls
                             need HWE_EULER.  0 = none (default) */
  int32_t pad_regions;
  hwe_region regions[HWE_MAX_REGIONS];
  double bstate[2][4];    /* states A and B of the prescribed kinds, conservative
                             variables (m of the 4 entries used) */
  double shock_x0;        /* HWE_BND_MOVING: switch position at t = 0 */
  double shock_speed;     /* and its speed in x */
  int32_t edge_rule;      /* Gauss-Legendre points per edge in the flux and
                             interface-value integrals of eqs. (fx)/(flux) and
                             (derave2d2): 2 (default; exact for cubics along the
                             edge) or 3 (exact for quintics); the positivity
                             limiter then checks the 9 points */
  int32_t pad_rule;
} hwe_opts;

/* Fill *o with the paper's defaults: linear weights 0.94/0.02/0.02/0.02
 * (Step 3), eps = 1e-8 (Step 5), gas_gamma = 1.4, adv = (1, 1), periodic unit
 * box, FP64, no limiter, device 0. */
hwe_status hwe_opts_default(hwe_opts* o);

/* Build a mesh handle (host FP64 precompute + one upload).
 *  nodes : host double [n_nodes][2] vertex coordinates
 *  tris  : host int32 [n_tris][3] vertex indices, any orientation
 *  Periodic meshes are tori: triangles may reference nodes across the seams
 *  and are unwrapped by minimal image about their first vertex.
 * Precomputes geometry, the Gauss-Legendre points of every edge (2, or 3 with
 * opts.edge_rule = 3), the face-neighbour stencils {K0, K1, K2, K3} of Step 1
 * (Fig. 1; ghost mirror cells on non-periodic boundaries), the boundary kind
 * of every boundary face (opts.walls, opts.regions) and, per cell, the linear
 * maps of the constrained least-squares problems of Steps 1 and 2.  Copies the inputs;
 * the caller keeps ownership.  Returns HWE_EMESH or HWE_ESINGULAR for bad
 * meshes, HWE_EHIP / HWE_ENOMEM for device failures, and HWE_EINVAL for a
 * device handle beyond the kernels' 32-bit indexing (N >= 2^28 cells, or
 * E >= 2^29 edges, 2^28 with the 3-point edge rule).  With a device it also
 * resolves the device address of the static scratch of hwe_step_noalloc.
 * *out is valid only on HWE_OK. */
hwe_status hwe_mesh_init(const double* nodes, int64_t n_nodes, const int32_t* tris, int64_t n_tris,
                         const hwe_opts* opts, hwe_mesh* out);

/* Release the handle and all its device memory (synchronises its device). */
hwe_status hwe_mesh_destroy(hwe_mesh m);

/* Sizes: number of cells N, edges E, and components m. Any pointer may be NULL. */
hwe_status hwe_mesh_info(hwe_mesh m, int64_t* n_cells, int64_t* n_edges, int32_t* m_comp);

/* perm_host[i] = caller's triangle index of internal cell i (host int64 [N]). */
hwe_status hwe_mesh_cell_perm(hwe_mesh m, int64_t* perm_host);

/* One explicit step of size dt (Sec. 2): reconstruction (Steps 1-6), the
 * Lax-Wendroff procedure and Taylor extrapolation at the edge Gauss points,
 * the space-time quadrature of the local Lax-Friedrichs flux (eqs. (fx),
 * (flux)), the update of eq. (flx) and the Green-Gauss derivative averages
 * (eqs. (derave2d2), (timeflux), (taylor2dtime)).
 *  wbar_in, grad_in   : device, state at t_n (layouts above); read only
 *  wbar_out, grad_out : device, state at t_n + dt; must not overlap the inputs
 * Time rule: 3-point Gauss-Lobatto (0, dt/2, dt; weights 1/6, 4/6, 1/6) whose
 * last node also gives the interface value of eq. (timeflux), or the option
 * of opts.time_rule; edge rule as opts.edge_rule.  Boundary states that move
 * with time are evaluated at (time set by hwe_set_time) + dt/2. */
hwe_status hwe_step(hwe_mesh m, const double* wbar_in, const void* grad_in, double* wbar_out,
                    void* grad_out, double dt, void* stream);

/* Vector-Jacobian product of hwe_step at the state (wbar_n, grad_n) with the
 * same dt (dt is a constant, not differentiated):
 *   (lam_wbar_n, lam_grad_n) = J(wbar_n, grad_n)^T (lam_wbar_np1, lam_grad_np1).
 * Same layouts and precision as hwe_step; outputs must not overlap inputs.
 * Non-smooth points: d|x| = sign(x) dx with sign(0) = 0; the max of the two
 * spectral radii in the flux viscosity takes the edge's first cell (the one
 * with the lower caller index) on ties.  Every boundary kind is
 * differentiated: a prescribed or moving boundary state is a constant of the
 * step (evaluated, as in hwe_step, at the time set by hwe_set_time + dt/2, so
 * set the time of step n before its adjoint), a reflective wall's exterior is
 * the mirrored interior.  The scaling limiter (opts.positivity = 1) is
 * differentiated on the branches the forward takes (the point of least
 * density, the point whose pressure root sets the scale); its threshold
 * eps = min(1e-13, rho_bar, p_bar) is a constant of the derivative. */
hwe_status hwe_step_adjoint(hwe_mesh m, const double* wbar_n, const void* grad_n,
                            const double* lam_wbar_np1, const void* lam_grad_np1, double* lam_wbar_n,
                            void* lam_grad_n, double dt, void* stream);

/* Reverse sweeps that recompute the forward states of a checkpoint segment
 * (Sec. 2 step, reversed by hwe_step_adjoint) can keep each step's
 * reconstruction (Steps 1-6) so that the adjoint does not rebuild it.
 *
 * hwe_step_keep: hwe_step whose reconstruction of the state at t_n is written
 * to recon_out and read from there by the step's edge stage (in place of the
 * handle's scratch).  Results are bitwise those of hwe_step.
 *  recon_out : device, caller-owned, [N][6][m] of double (FP64) or float
 *              (MIXED): per cell and component the coefficients a0..a5 of
 *              R - Wbar in the monomial basis about the cell centroid (the
 *              layout of hwe_debug_recon); 16-byte aligned (it is read as
 *              whole 16-byte records); must not overlap the state buffers.
 *
 * hwe_step_adjoint_kept: hwe_step_adjoint with recon_n = the buffer that
 * hwe_step_keep wrote for the same (wbar_n, grad_n) on this handle; the
 * reconstruction launch is skipped and the result is bitwise that of
 * hwe_step_adjoint.  The library cannot check that recon_n belongs to the
 * state: a buffer from another state gives a wrong product without an error.
 * Both return HWE_EINVAL for a null recon buffer and under the conditions of
 * the calls they extend. */
hwe_status hwe_step_keep(hwe_mesh m, const double* wbar_in, const void* grad_in, double* wbar_out,
                         void* grad_out, double dt, void* recon_out, void* stream);
hwe_status hwe_step_adjoint_kept(hwe_mesh m, const double* wbar_n, const void* grad_n, const void* recon_n,
                                 const double* lam_wbar_np1, const void* lam_grad_np1, double* lam_wbar_n,
                                 void* lam_grad_n, double dt, void* stream);

/* For callers that cannot allocate device memory when they step: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 *
 * hwe_step_noalloc: hwe_step whose scratch (the reconstruction, [N][6][m] of
 * double or float by precision, the edge fluxes, [E][m] double, and the
 * interface values, [E][m] double or float, each part 256-byte aligned) lives
 * in one static device array of HWE_NOALLOC_SCRATCH_BYTES per GPU that the
 * library holds until the process ends, in place of the handle's scratch.  It
 * calls no hipMalloc, hipFree or allocating library routine.  The array's
 * device address is resolved by hwe_mesh_init for the handle's device.
 * Same arguments, checks and results (bitwise) as hwe_step.
 *  - HWE_EINVAL if the mesh's scratch exceeds HWE_NOALLOC_SCRATCH_BYTES
 *    (64 MiB: e.g. 204,800 Euler triangles in FP64 need 59.0 MB, in the mixed
 *    precision 39.3 MB); the message gives both sizes.
 *  - Every call on one GPU, from any handle or thread, shares that GPU's
 *    array, which keeps the last call's contents: calls that overlap in time
 *    on one GPU race (serialise them, e.g. on one stream).  Nothing in the
 *    array needs clearing: a step writes every entry it reads before reading
 *    it. */
#define HWE_NOALLOC_SCRATCH_BYTES (64u << 20)
hwe_status hwe_step_noalloc(hwe_mesh m, const double* wbar_in, const void* grad_in, double* wbar_out,
                            void* grad_out, double dt, void* stream);

/* Time of the state handed to the following hwe_step / hwe_step_keep /
 * hwe_step_adjoint / hwe_step_adjoint_kept calls on this handle (default 0).  Only HWE_BND_MOVING faces depend on it: a step
 * from time t with size dt evaluates them at t + dt/2.  Host-side; the value is
 * taken when a step is launched. */
hwe_status hwe_set_time(hwe_mesh m, double t);

/* Step size of the time loop.  Sec. 3 fixes only the CFL number (0.5 there);
 * the length and speed it scales are a reading: dt = cfl * min_K r_K /
 * max_K lambda_K with r_K the inradius of K and lambda_K the largest signal
 * speed over all directions at the cell average (|a| for advection,
 * sqrt(2)|u| for Burgers, |(u, v)| + c for Euler).  Writes one double to
 * device memory dt_dev; a NaN average gives a NaN step. */
hwe_status hwe_max_dt(hwe_mesh m, const double* wbar, double cfl, double* dt_dev, void* stream);

/* State diagnostics into device int32 flags_dev[1] (overwritten):
 * bit 0 = a non-finite cell average, bit 1 = density <= 0, bit 2 = pressure <= 0
 * (bits 1-2 for Euler only). */
hwe_status hwe_check_state(hwe_mesh m, const double* wbar, int32_t* flags_dev, void* stream);

/* Reconstruction only (Steps 1-6) for kernel-level tests: R_out is device
 * [N][6][m] (internal cell order) of double (FP64) or float
 * (MIXED) holding, per cell and component, the coefficients a0..a5 of R - Wbar
 * in the monomial basis about the cell centroid:
 * R(x,y) - Wbar = a0 + a1 X + a2 Y + a3 X^2 + a4 XY + a5 Y^2.
 * Moving boundary states are taken at the time set by hwe_set_time (a step
 * takes them at that time + dt/2).  R_out must be 16-byte aligned (whole
 * records are written with 16-byte stores); HWE_EINVAL if it is not or if it
 * overlaps the state. */
hwe_status hwe_debug_recon(hwe_mesh m, const double* wbar, const void* grad, void* R_out, void* stream);

/* Edge stage only (Sec. 2.1, eqs. (fx), (flux), (tay), (tayext), and the
 * interface value of eq. (timeflux)) for kernel-level tests, from a
 * reconstruction R in the layout of hwe_debug_recon and the cell averages
 * wbar of the same state, with step size dt:
 *  F_out : device double [E][m]: |e| times the time and Gauss-point average of
 *          the local Lax-Friedrichs normal flux through edge e, oriented out of
 *          its first cell (hwe_debug_host_array 8); the first cell's average
 *          changes by -dt/|K| F_e, the second's by +dt/|K| F_e (eq. (flx));
 *  G_out : device [E][m] of double (FP64) or float (MIXED): the Gauss-point
 *          average of the two sides' offsets W - Wbar at t_n + dt, halved, so
 *          that the interface value at the edge is (Wbar_1 + Wbar_2)/2 + G_e.
 * Edges are in the library's order; hwe_debug_host_array 7 gives each cell's
 * edges.  R, F_out and G_out must be 16-byte aligned (whole records are moved
 * with 16-byte accesses); outputs must not overlap the inputs or each other. */
hwe_status hwe_debug_edge(hwe_mesh m, const void* R, const double* wbar, double dt, double* F_out, void* G_out,
                          void* stream);

/* Host copy of a precomputed per-cell array for host-logic tests (works for
 * host-only handles).  which: 0 = p1 map [55][N] (rows: c1..c5 of the
 * zero-mean basis X, Y, X^2-Mxx, XY-Mxy, Y^2-Myy; columns: dW1..dW3, V0..V3,
 * Y0..Y3), 1 = centroid [2][N], 2 = area [N], 3 = moments [3][N],
 * 4 = neighbours [3][N] (as double; negative = boundary), 5 = boundary kind
 * of each face [3][N] (hwe_bnd_kind as double; -1 = interior face), 6 = the
 * factored p1 map of the device tables [41][N] (rows 3j + c: the dW columns;
 * 15 + 5k + j: Z; 25 + 8k + v: Q on V0..V3, Y0..Y3; the map's V and Y columns
 * are Z^T Q), 7 = each cell's edges [3][N] (edge index << 1 | 1 when the cell
 * is the edge's second cell), 8 = each edge's cells [2][E] (first, second; a
 * negative second entry marks a boundary edge).  out is host double with room
 * for the stated size. */
hwe_status hwe_debug_host_array(hwe_mesh m, int32_t which, double* out);

/* Per-kernel timing for measurement tools.  hwe_profile_begin arms HIP events
 * around the three kernels of the next n_steps calls of hwe_step on this
 * handle (the events are recorded on each call's stream; no synchronisation
 * inside hwe_step).  hwe_profile_end synchronises on the recorded events and
 * returns in ms_sum[3] the summed durations in milliseconds of the
 * reconstruction, edge and update kernels, and in *n_steps_done the number of
 * profiled steps; it disarms profiling. */
hwe_status hwe_profile_begin(hwe_mesh m, int32_t n_steps);
hwe_status hwe_profile_end(hwe_mesh m, double* ms_sum, int32_t* n_steps_done);

/* Thread-local message for the last failing call on this thread. */
const char* hwe_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HWE_H */
