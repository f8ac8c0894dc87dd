/*
 * libugks -- MI355X (gfx950) implementation of one dual-time pseudo-iteration
 * of the implicit unsteady unified gas-kinetic scheme (UGKS) on moving
 * overset structured meshes, after Zhang, Long, Cao, Xu, "Unified Gas-Kinetic
 * Scheme for Unsteady Multiscale Flows with Moving Boundaries".
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Return value: UGKS_OK (0) or a negative UGKS_E_* code; ugks_last_error()
 *    returns a thread-local message for the last failure.  Arguments are
 *    validated before anything is launched, so on error nothing is written.
 *    No C++ exception crosses this interface.
 *  - Device arrays are caller-owned HIP device pointers; the library never
 *    frees them.  Host arrays are marked "host".  The context owns its own
 *    device copies of the geometry; its scratch (and the reverse mode's
 *    workspace) is its own allocation or a caller's workspace
 *    (ugks_workspace_size, ugks_create_with_workspace).
 *  - Every compute call is asynchronous on `stream` (a hipStream_t passed as
 *    void*, NULL = the null stream).  Calls on one context must not overlap.
 *  - Layouts.  nv = nvx*nvy discrete velocities, k = ix + nvx*iy.  The reduced
 *    distributions h, b (Sec. 2.1: h = int f dxi, b = int xi^2 f dxi) and the
 *    arrays of the same shape (sources, divergences) are [ncell][nv],
 *    velocity innermost, in the storage type chosen at creation (double for
 *    UGKS_F64, float for UGKS_F32).  W is [ncell][dim+2] (rho, rho U, rho E)
 *    and q [ncell][dim], always double.  Face arrays are [nface][...].
 *  - Cells are numbered block by block, i fastest (cell0(b) + i + ni*j).
 *    Faces: per block first the i-faces ((ni+1)*nj, index i + (ni+1)*j, face
 *    i lies on the low-i side of cell i), then the j-faces (ni*(nj+1)).  A
 *    face's normal points from its low-index side to its high-index side.
 *  - Monatomic gas (no internal degrees of freedom): b carries the 3-dim
 *    velocity components that the dim-dimensional grid does not resolve.
 */
#ifndef UGKS_H
#define UGKS_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define UGKS_OK 0
#define UGKS_E_ARG (-1)         /* null pointer or value out of range */
#define UGKS_E_SHAPE (-2)       /* inconsistent sizes */
#define UGKS_E_DEVICE (-3)      /* a HIP call failed */
#define UGKS_E_NONPHYS (-4)     /* non-positive density or temperature */
#define UGKS_E_ORPHAN (-5)      /* a receptor cell found no donor */
#define UGKS_E_UNSUPPORTED (-6) /* feature not available for this input */

/* storage precision of h, b and the arrays of their shape */
#define UGKS_F64 0 /* double storage, double arithmetic */
#define UGKS_F32 1 /* float storage and float flux arithmetic; moments,
                      the equilibrium solve and residual assembly in double */

/* block side kinds (sides: 0 i-min, 1 i-max, 2 j-min, 3 j-max) */
#define UGKS_BC_PERIODIC 0 /* both sides of a direction */
#define UGKS_BC_FARFIELD 1 /* ghost = Maxwellian of the far-field state */
#define UGKS_BC_COPY 2     /* ghost = adjacent cell (zero gradient) */
#define UGKS_BC_WALL 3     /* diffuse isothermal wall (Eq. maxWalldes) */
#define UGKS_BC_NONE 4     /* overset fringe: no face */

/* cell kinds */
#define UGKS_HOLE 0
#define UGKS_FIELD 1
#define UGKS_RECEPTOR 2

/*
 * Problem statement (Sec. 2.1 kinetic model and discretisation; Sec. 3 mesh).
 * All pointers are host pointers, read during ugks_create only.
 *   dim            1 or 2.
 *   pr, omega      Prandtl number of the Shakhov model; viscosity exponent.
 *   mu_ref, rt_ref collision time tau = mu_ref (RT/rt_ref)^omega / p;
 *                  mu_ref <= 0 means collisionless (1/tau = 0).
 *   nvx, nvy, vx, vy, vrange
 *                  uniform velocity points per axis on [vrange[0], vrange[1]]
 *                  x [vrange[2], vrange[3]] (nvy = 1, vy = {0} in 1D);
 *                  weights are composite closed Newton-Cotes per axis.
 *   winf           far-field conservative state (dim+2 values).
 *   cfl_s, cfl_p   CFL of the explicit flux step dt_s and of the virtual
 *                  step dt' (the paper uses 0.5 and 100).
 *   nblock, bint   per block 6 ints: ni, nj (1 in 1D), bc[4].
 *   bdbl           per block 14 doubles: wall RT per side (4), wall velocity
 *                  added to the mesh velocity per side (x: 4, y: 4), and the
 *                  rotation centre at the reference pose (2).
 *   nodes          per block the reference node coordinates, x then y, each
 *                  (ni+1)*(nj+1) values with index i + (ni+1)*j (1D: x only).
 *   prec           UGKS_F64 or UGKS_F32.
 *   nvu, vu, wu    optional unstructured velocity mesh (2D; nvu = 0: the
 *                  uniform grid above).  nvu > 0 replaces it by nvu points
 *                  vu (x components, then y components) with weights wu,
 *                  the areas of their velocity cells (Sec. 2.1: V_k is the
 *                  volume of the k-th velocity cell); nvx, nvy, vx, vy and
 *                  vrange are then ignored.  UGKS_E_ARG for a non-positive
 *                  weight or a null array, UGKS_E_UNSUPPORTED in 1D.
 */
typedef struct {
  int32_t dim;
  double pr, omega, mu_ref, rt_ref;
  int32_t nvx, nvy;
  const double* vx;
  const double* vy;
  double vrange[4];
  double winf[4];
  double cfl_s, cfl_p;
  int32_t nblock;
  const int32_t* bint;
  const double* bdbl;
  const double* nodes;
  int32_t prec;
  int32_t nvu;
  const double* vu;
  const double* wu;
} ugks_problem;

typedef struct ugks_ctx ugks_ctx;

/* Create a context on HIP device `device`: copies the problem, builds the
   geometry at the reference pose, uploads it and allocates scratch.
   *out receives the context.  Block sizes the sweeps accept (one workgroup
   per block and velocity chunk, state in LDS): nj <= 512 in 2D; ni <= 256
   when a block is periodic in j; the LU-SGS sweeps' LDS of the largest
   block within 160 KiB, which bounds nj to 511 (else UGKS_E_UNSUPPORTED,
   with the reason in ugks_last_error). */
int ugks_create(const ugks_problem* p, int device, ugks_ctx** out);
/*
 * Device memory a problem needs beyond the caller's state arrays (host
 * outputs, either may be NULL): *scratch receives the bytes of the
 * context's scratch (face and cell records, W gradients, chunk partial
 * sums of the face moments and macro fluxes, the macro and micro LU-SGS
 * intermediates: Secs. 2.1-2.2), *adjoint the bytes of the reverse-mode
 * workspace (about 14 FP64 arrays of [ncell][nv]).  The geometry and table
 * copies a context keeps (O(ncell + nface)) are not included.  UGKS_E_ARG
 * or UGKS_E_SHAPE for a problem ugks_create would reject on those grounds.
 */
int ugks_workspace_size(const ugks_problem* p, size_t* scratch, size_t* adjoint);

/*
 * ugks_create with a caller-owned device workspace `work` of work_bytes
 * (256-byte aligned; at least the scratch bytes of ugks_workspace_size):
 * the context's scratch lives there instead of in its own allocation, and
 * when work_bytes also covers the adjoint bytes (scratch + adjoint) the
 * reverse-mode workspace follows the scratch in it, so that neither the
 * step nor the adjoint allocates device memory.  The workspace must outlive
 * the context; the library never frees it.  UGKS_E_SHAPE if it is too small.
 */
int ugks_create_with_workspace(const ugks_problem* p, int device, void* work, size_t work_bytes, ugks_ctx** out);

/* Release the context and its device memory.  NULL is accepted. */
int ugks_destroy(ugks_ctx* ctx);
/* Sizes: cells, faces, velocities, storage precision (any pointer may be NULL). */
int ugks_sizes(const ugks_ctx* ctx, int32_t* ncell, int32_t* nface, int32_t* nv, int32_t* prec);

/*
 * Rigid motion of every block to the poses of the next physical time
 * (Sec. 3, Step 1): host array poses[nblock][6] = translation (dx, dy),
 * rotation th about the moved centre, velocity (ux, uy), angular velocity om.
 * Recomputes node positions, cell and face geometry, the face grid velocity
 * U_f = u + om x (x_f - centre), the explicit flux step dt_s (written to
 * *dts, host) and the per-cell virtual steps dt', and uploads them.  The
 * geometry is frozen until the next call (both flux levels of a physical
 * step use it).  Synchronous.
 */
int ugks_set_poses(ugks_ctx* ctx, const double* poses, double* dts);

/* Host cell kinds [ncell] (UGKS_HOLE / FIELD / RECEPTOR); default all field. */
int ugks_set_types(ugks_ctx* ctx, const int8_t* types);
int ugks_get_types(const ugks_ctx* ctx, int8_t* types);

/*
 * Overset donor table (Sec. 3.2), host CSR: receptor cells rec[nrec], donors
 * of receptor r are don[ptr[r] .. ptr[r+1]-1] with weights w (sum to 1).
 * Donors must be field cells.  Copied to the device.
 */
int ugks_set_overset(ugks_ctx* ctx, int32_t nrec, const int32_t* rec, const int32_t* ptr,
                     const int32_t* don, const double* w);

/*
 * Overset assembly at the current geometry (Sec. 3.1, host; 2D): each block
 * is a grid zone.  A node is inactive inside another zone's body (closed
 * wall outline) or where another zone has a cell containing it, at least
 * overlap+3 cell layers inside that zone's overset (UGKS_BC_NONE) sides,
 * and a nearer wall (ties: the higher zone).  Cells: field (all nodes
 * active), hole (none active), else boundary; receptors = boundary cells,
 * one buffer layer of field cells beside boundary or hole cells, and
 * `overlap` layers beside overset sides.  Donor (Sec. 3.2): the field cell
 * of another zone containing the receptor centroid (lowest zone, then
 * lowest cell).  Weights, wrule 0: inverse distance squared over the donor
 * and its field index neighbours; wrule 1: bilinear over the quad of
 * donor-grid centroids around the receptor (inverse distance where no such
 * quad of field cells contains it).  Installs the cell kinds and the donor
 * table; *nrec receives the receptor count.  UGKS_E_ORPHAN if a receptor has
 * no donor, UGKS_E_ARG for wrule not 0/1 or overlap < 0, UGKS_E_UNSUPPORTED
 * in 1D; nothing is installed on error.  Synchronous.
 */
int overset_assemble(ugks_ctx* ctx, int32_t wrule, int32_t overlap, int32_t* nrec);
/*
 * overset_assemble on the context's GPU (Secs. 3.1-3.2): bins of each zone's
 * cells, node classes one thread per node, cell kinds and receptor layers
 * one thread per cell, donors and weights one thread per receptor, rows
 * compacted by scans; the same predicates and arithmetic without
 * contraction, so kinds, receptors, donors and weights equal
 * overset_assemble's bit for bit.  Same arguments, errors and installation;
 * uses temporary device memory and a stream of its own; synchronous.
 */
int overset_assemble_device(ugks_ctx* ctx, int32_t wrule, int32_t overlap, int32_t* nrec);

/* The installed donor table (host copies): *nrec receptors, *ndon donor
   entries; rec[nrec], ptr[nrec+1], don[ndon], w[ndon] are filled when not
   NULL (call once with NULL arrays to read the sizes). */
int ugks_get_overset(const ugks_ctx* ctx, int32_t* nrec, int32_t* ndon, int32_t* rec, int32_t* ptr,
                     int32_t* don, double* w);

/* Discrete reduced Maxwellian h = H(W), b = B(W) at every cell
   (initialisation). */
int ugks_maxwellian(ugks_ctx* ctx, const double* W, void* h, void* b, void* stream);

/*
 * Velocity moments (Sec. 2.1): W = sum_k V_k Psi_k (h, b) and the heat flux
 * q = 1/2 sum_k V_k c (|c|^2 h + b), c = v_k - U of that W, for every cell.
 */
int ugks_moments(ugks_ctx* ctx, const void* h, const void* b, double* W, double* q, void* stream);

/*
 * Heat flux q = 1/2 sum_k V_k c (|c|^2 h + b) with c = v_k - U, U the
 * velocity of the given W (Sec. 2.1 moments), for every non-hole cell.
 * This is the q that the Shakhov equilibrium of (W, q) uses.
 */
int ugks_heatflux(ugks_ctx* ctx, const void* h, const void* b, const double* W, double* q, void* stream);

/*
 * UGKS flux (Sec. 2.1, Eqs. microscopicFlux, macroscopicFlux, fullSolution,
 * maxWalldes; time-averaged over dt_s as in Sec. 2.2) of the state (h, b, W,
 * q): divergence Dh, Db [ncell][nv] = -(1/|Omega_i|) sum_f sigma S_f F_f,k
 * (zero on non-field cells), face macro flux F [nface][dim+2] along the face
 * normal, and wall output wall [nface][dim+3] = (rho_w, macro flux into the
 * wall) on wall faces (zero elsewhere).  F and wall may be NULL.
 */
int ugks_flux(ugks_ctx* ctx, double dts, const void* h, const void* b, const double* W,
              const double* q, void* Dh, void* Db, double* F, double* wall, void* stream);

/*
 * ugks_flux for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation):
 * the same operation and results as ugks_flux, with its scratch (W
 * gradients, face records, per-chunk partial sums, and the face macro flux
 * when F is NULL) in the library's file-scope static device array of
 * 128 MiB instead of the context's buffers.  Calls no allocating routine.
 * UGKS_E_SHAPE (nothing launched) when the case needs more than the array:
 * 8 ncell + 40 nface + 9 nface ceil(nv/64) (+ (dim+2) nface with F NULL)
 * doubles, each part rounded up to 256 bytes.  Every call on a device
 * shares that device's array, which keeps the last call's contents (the
 * face records are cleared on entry): calls that overlap on one device,
 * on any stream or context, race.
 */
int ugks_flux_noalloc(ugks_ctx* ctx, double dts, const void* h, const void* b, const double* W, const double* q,
                      void* Dh, void* Db, double* F, double* wall, void* stream);

/* Overset interpolation (Sec. 3.2) of h, b, W and q into the receptor rows,
   in place. */
int overset_interp(ugks_ctx* ctx, void* h, void* b, double* W, double* q, void* stream);

/*
 * Steps 1-2 of the dual time stepping (Sec. 2.2): interpolate receptors,
 * evaluate the level-n flux and store the source S = f^n/dt + r^n/2 with
 * r^n of Eq. residual_macro_n (Sh, Sb [ncell][nv]) and the level-n face
 * flux Fn [nface][dim+2].  q [ncell][dim] is the heat flux of f^n about
 * the velocity of W^n (as ugks_heatflux returns); receptor rows of h, b, W, q
 * are refreshed by interpolation, and so, once after an overset_assemble,
 * are the cells that were holes and are field cells now (their data is
 * stale: they are filled by the same donor rule).
 */
int ugks_begin_step(ugks_ctx* ctx, double dt, void* h, void* b, double* W, double* q,
                    void* Sh, void* Sb, double* Fn, void* stream);

/*
 * Steps 3-7 of the dual time stepping, n_inner times (Sec. 2.2): per inner
 * iteration interpolate receptors, evaluate the flux, solve the macro delta
 * form (Eq. dualTimeStepping_macro) by LU-SGS, solve the micro delta form
 * (Eq. dualTimeStepping_micro) by LU-SGS per velocity and correct W
 * (Step 7).  Wn is W at level n.  resid (device, may be NULL) receives
 * [n_inner][dim+2] L2 norms of the macro residual over field cells.
 * Failures found on the device (see ugks_status) are returned here only in
 * the synchronising check mode of ugks_set_checks.
 */
int ugks_step(ugks_ctx* ctx, double dt, int32_t n_inner, void* h, void* b, double* W,
              const double* Wn, double* q, const void* Sh, const void* Sb, const double* Fn,
              double* resid, void* stream);

/*
 * Instrumented ugks_step for measurement: the same n_inner pseudo-iterations,
 * with HIP events recorded on `stream` between the kernels; waits for the
 * last event and writes host stage_ms[UGKS_NSTAGE], the mean milliseconds
 * per pseudo-iteration of: 0 overset interpolation, 1 W gradients and wall
 * incident states, 2 face-moment pass (the face-equilibrium march kernel;
 * 1D: the face-equilibrium kernel), 3 face-equilibrium finalize, 4 flux
 * pass (the flux march kernel; 1D: the flux kernel), 5 flux finalize,
 * 6 macro LU-SGS, 7 cell equilibrium records, 8 micro residual pass,
 * 9 micro LU-SGS sweeps, 10 Step-7 moments.
 */
#define UGKS_NSTAGE 11
int ugks_step_profile(ugks_ctx* ctx, double dt, int32_t n_inner, void* h, void* b, double* W,
                      const double* Wn, double* q, const void* Sh, const void* Sb, const double* Fn,
                      double* stage_ms, void* stream);

/* Current explicit flux step dt_s and a copy of the virtual steps dt' (host
   array [ncell], may be NULL). */
int ugks_timesteps(const ugks_ctx* ctx, double* dts, double* dtp);

/*
 * Replayed pseudo-iterations: the same work as ugks_step (Sec. 2.2, Steps
 * 3-7, n_inner >= 1 times), captured once into a HIP graph on a private
 * stream and launched on `stream`.  The graph is kept by the context and
 * captured again when dt, n_inner, any array pointer, the geometry, the
 * cell kinds, the donor table or the launch shapes change (an update of the
 * executable graph in place when possible).  Results are identical to
 * ugks_step.  Not thread-safe per context.
 */
int ugks_step_graph(ugks_ctx* ctx, double dt, int32_t n_inner, void* h, void* b, double* W, const double* Wn,
                    double* q, const void* Sh, const void* Sb, const double* Fn, double* resid, void* stream);

/*
 * Batches of independent cases (ragged sizes, one context each, all on one
 * device): ugks_batch_step runs n_inner pseudo-iterations (Sec. 2.2,
 * Steps 3-7) of every case from one captured graph launched on `stream`.
 * Array arguments are host arrays of ncase device pointers in case order
 * (resid may be NULL, or hold NULL entries).  Cached like ugks_step_graph
 * (the first call after a change of the arguments, the cases' geometry or
 * donor tables waits for the device and rebuilds the graph); results are
 * identical to ugks_step per case, bit for bit.  The batch keeps the
 * context pointers: destroy it before them.
 *
 * Mode 1 (the default where it applies: 2D cases of one storage type): one
 * launch per stage of the pseudo-iteration for all cases; the per-cell and
 * per-face stages run one grid over every case's cells or faces, and the
 * two march passes and the micro LU-SGS sweep run persistent grids that
 * stride over (case, velocity chunk, row group or block) work items, the
 * costliest first.  Mode 0: each case's own kernel chain, the chains on up
 * to four concurrent branches (round robin over the cases).
 * ugks_batch_set_mode returns UGKS_E_UNSUPPORTED for mode 1 on other
 * batches, UGKS_E_ARG for another mode; ugks_batch_get_mode gives the mode
 * in effect.
 */
typedef struct ugks_batch ugks_batch;
int ugks_batch_create(int32_t ncase, ugks_ctx* const* ctxs, ugks_batch** out);
int ugks_batch_step(ugks_batch* batch, const double* dt, int32_t n_inner, void* const* h, void* const* b,
                    double* const* W, const double* const* Wn, double* const* q, const void* const* Sh,
                    const void* const* Sb, const double* const* Fn, double* const* resid, void* stream);
int ugks_batch_set_mode(ugks_batch* batch, int32_t mode);
int ugks_batch_get_mode(const ugks_batch* batch, int32_t* mode);
int ugks_batch_destroy(ugks_batch* batch);

/*
 * Launch shapes (results do not depend on them): kc_max, the widest velocity
 * chunk of a micro-sweep workgroup (16, 8 or 4; narrowed for tall blocks),
 * and rg_eq, rg_flux, the core rows per workgroup of the face-equilibrium
 * and flux march kernels (10, 8 or 6 each).  ugks_autotune times n_inner
 * pseudo-iterations run on device copies of the given state (the caller's
 * arrays are not written) for kc_max
 * {16, 8, 4}, then rg_eq {8, 10, 6} and then rg_flux {8, 10, 6}, each with the
 * others at their best so far (the three act on different kernels), keeps
 * the fastest and reports it in host choice[3] and its mean milliseconds per
 * pseudo-iteration in *best_ms.  The state copies live in the reverse-mode
 * workspace when the context has one, else they are allocated for the call.
 * Synchronous.
 */
int ugks_set_tuning(ugks_ctx* ctx, int32_t kc_max, int32_t rg_eq, int32_t rg_flux);
int ugks_get_tuning(const ugks_ctx* ctx, int32_t* kc_max, int32_t* rg_eq, int32_t* rg_flux);
/*
 * The micro sweep's launch under the current kc_max (host outputs, any may
 * be NULL): velocity-chunk width, rows per thread, depth of the register ring
 * of prefetched hyperplanes, and 1 when the micro residual (Eq.
 * residual_micro_n+1,s) is formed inside the forward sweep instead of by a
 * separate pass (2D, one row per thread and chunks of 8 or 16 velocities).
 * Results do not depend on it.  Returns UGKS_E_ARG for a NULL context.
 */
int ugks_micro_shape(const ugks_ctx* ctx, int32_t* kc, int32_t* rows, int32_t* depth, int32_t* fused);
int ugks_autotune(ugks_ctx* ctx, double dt, int32_t n_inner, const void* h, const void* b, const double* W,
                  const double* Wn, const double* q, const void* Sh, const void* Sb, const double* Fn,
                  int32_t* choice, double* best_ms, void* stream);

/*
 * Wall temperature (Eq. maxWalldes): RT of the isothermal wall on side
 * `side` (0 i-min, 1 i-max, 2 j-min, 3 j-max) of block `blk`; updates the
 * face data of that side.  UGKS_E_ARG for a bad block, side or rtw <= 0.
 */
int ugks_set_wall_rt(ugks_ctx* ctx, int32_t blk, int32_t side, double rtw);

/*
 * Far-field state (Sec. 2.1: far-field sides take the Maxwellian of a given
 * state as their ghost distribution): winf (host, D + 2 conservative
 * values rho, rho u, [rho v,] rho E) replaces the state of ugks_problem and
 * its Maxwellian from the next call on, e.g. to ramp an inflow.  Waits for
 * the device first.  UGKS_E_ARG for a null pointer, a non-finite value or
 * a non-positive density or internal energy.
 */
int ugks_set_farfield(ugks_ctx* ctx, const double* winf);

/*
 * Rigid velocity (ux, uy) and angular velocity om of block `blk` at the
 * current node positions (the prescribed body motion of Sec. 3): face grid
 * velocities U_f and wall velocities are recomputed; node positions, dt_s and
 * the virtual steps dt' stay those of the last ugks_set_poses.  Synchronous.
 */
int ugks_set_block_velocity(ugks_ctx* ctx, int32_t blk, double ux, double uy, double om);

/* Host copy of the face data [nface][8]: unit normal (x, y; from the low to
   the high cell of the face), area, grid velocity (x, y), wall velocity
   (x, y) and wall RT (wall faces; zero elsewhere). */
int ugks_face_geometry(const ugks_ctx* ctx, double* fgeo);

/* Rows of the installed donor table: receptors, rows of the cells uncovered
   from holes by the last overset_assemble, and whether those are still to be
   filled by the next ugks_begin_step (1) or not (0). */
int ugks_overset_rows(const ugks_ctx* ctx, int32_t* nrec, int32_t* nrefill, int32_t* pending);

/* Device copy of the face macro flux F [nface][dim+2] of the last flux
   evaluation (Step 3 of the last pseudo-iteration run by ugks_step,
   ugks_step_graph or ugks_step_adjoint's recomputation, or ugks_flux). */
int ugks_last_flux(const ugks_ctx* ctx, double* F, void* stream);

/*
 * Reverse mode (hand-written adjoint, vector-Jacobian products) of the
 * dual-time stepping, for FP64 contexts in 2D (else UGKS_E_UNSUPPORTED).
 * "x_bar" is the cotangent of x: a device FP64 array in x's layout; output
 * cotangents of the map are inputs (NULL means zero), input cotangents are
 * written (not accumulated).  face_bar (may be NULL) receives [nface][5]:
 * the cotangents of the face grid velocity U_f (x, y; Eq. BGK w = v - U),
 * of the wall velocity (x, y) and of the wall RT (Eq. maxWalldes) of each
 * face, so that a rigid body velocity's gradient is the sum of the U_f and
 * wall-velocity entries over the body's faces, and a wall temperature's the
 * sum of the RT entries over its faces.  Node positions, cell kinds, donor
 * tables, dt, dt_s and dt' are held fixed.  At the method's kinks (limiter
 * switches, upwind sign, positivity fallbacks, |.| of the spectral radius)
 * the derivative of the branch the forward pass takes is returned.  Each
 * call recomputes the forward quantities it needs from the given inputs
 * (the inputs are not modified) in its FP64 workspace (about 14 arrays of
 * [ncell][nv]: the caller's, see ugks_create_with_workspace, or allocated
 * on first use); the context's scratch is overwritten.  Every bar is summed
 * in an order fixed by the mesh (the scatters run over write-disjoint
 * colourings of faces, cells and donor rows, computed on the host when the
 * tables change and kept in the workspace), so the results are bitwise
 * reproducible from call to call and across contexts.
 * The cotangent of a hole cell's value is not defined.  Asynchronous on
 * `stream`.
 *
 * ugks_flux_adjoint: the map (h, b, W, q) -> (Dh, Db, F) of ugks_flux at
 * dt_s (Sec. 2.1, Eqs. microscopicFlux, macroscopicFlux, fullSolution,
 * maxWalldes).
 */
int ugks_flux_adjoint(ugks_ctx* ctx, const void* h, const void* b, const double* W, const double* q,
                      const double* Dh_bar, const double* Db_bar, const double* F_bar, double* h_bar,
                      double* b_bar, double* W_bar, double* q_bar, double* face_bar, void* stream);

/*
 * One inner iteration (Sec. 2.2, Steps 3-7; ugks_step with n_inner = 1)
 * reversed: the map (h, b, W, q; Wn, Sh, Sb, Fn) -> (h', b', W', q'; F) at
 * the given inputs, F being the face macro flux of its Step 3 (as
 * ugks_last_flux returns).  Output cotangents h1_bar, b1_bar [ncell][nv],
 * W1_bar [ncell][dim+2], q1_bar [ncell][dim], F_bar [nface][dim+2]; input
 * cotangents h_bar, b_bar, W_bar, Wn_bar, q_bar, Sh_bar, Sb_bar, Fn_bar.
 */
int ugks_step_adjoint(ugks_ctx* ctx, double dt, const void* h, const void* b, const double* W, const double* Wn,
                      const double* q, const void* Sh, const void* Sb, const double* Fn, const double* h1_bar,
                      const double* b1_bar, const double* W1_bar, const double* q1_bar, const double* F_bar,
                      double* h_bar, double* b_bar, double* W_bar, double* Wn_bar, double* q_bar,
                      double* Sh_bar, double* Sb_bar, double* Fn_bar, double* face_bar, void* stream);

/*
 * Steps 1-2 (ugks_begin_step) reversed: the map (h, b, W, q) -> (h', b', W',
 * q'; Sh, Sb, Fn), the primed state being the input with its receptor rows
 * (and, with refill != 0, first the rows of the cells uncovered from holes
 * by the last overset_assemble) interpolated.  refill must say whether the
 * forward call filled those cells (ugks_begin_step does once after an
 * assembly); the donor table must be the one that call used.
 */
int ugks_begin_step_adjoint(ugks_ctx* ctx, double dt, const void* h, const void* b, const double* W,
                            const double* q, int32_t refill, const double* h1_bar, const double* b1_bar,
                            const double* W1_bar, const double* q1_bar, const double* Sh_bar,
                            const double* Sb_bar, const double* Fn_bar, double* h_bar, double* b_bar,
                            double* W_bar, double* q_bar, double* face_bar, void* stream);

/*
 * Device-side checks.  Kernels record failures in the context's status
 * word: the micro LU-SGS sweep (Eq. dualTimeStepping_micro) when its bounded
 * wait for a neighbouring wavefront runs out (it then goes on, so the kernel
 * ends, but the f it writes is not valid), and Step 7 (Sec. 2.2) when the
 * corrected W of a field cell has a non-positive density or temperature or
 * a non-finite entry.  ugks_status waits for `stream`, reads and clears the
 * word and returns UGKS_E_DEVICE (wait ran out; checked first),
 * UGKS_E_NONPHYS, or UGKS_OK.
 */
int ugks_status(ugks_ctx* ctx, void* stream);
/*
 * sync != 0: ugks_begin_step, ugks_step and ugks_step_graph wait for their
 * stream at the end and return ugks_status (default 0: asynchronous, the
 * status is read by an explicit ugks_status).  wait_limit >= 0 sets the
 * bound of the micro sweep's neighbour wait in sleeps (default 2^20, also
 * for a negative value); a small bound lets a test force the failure path.
 */
int ugks_set_checks(ugks_ctx* ctx, int32_t sync, int32_t wait_limit);

/*
 * Wall loads (Sec. 2.1: the macro flux into an isothermal wall, Eq.
 * maxWalldes; the load and heat flux on a body) from a face macro flux F
 * [nface][dim+2] (ugks_flux, ugks_last_flux).  face_loads [nface][dim+3]
 * (device, may be NULL): per wall face the momentum flux into the wall per
 * unit area (dim components: the load on the body per area), its component
 * along the normal pointing into the wall (pressure p_w) and along that
 * normal turned by +90 degrees (shear sigma_w; 0 in 1D), and the energy flux
 * into the wall q_w; zero on faces that are not walls.  side_loads
 * [nblock][4][4] (device, may be NULL): per block side (0 i-min, 1 i-max,
 * 2 j-min, 3 j-max) the area integrals of the force on the body (x, y), of
 * its moment about the block's moved rotation centre (z) and of q_w; zero
 * on sides that are not walls.  Sums run in face order (reproducible).
 */
int ugks_wall_loads(ugks_ctx* ctx, const double* F, double* face_loads, double* side_loads, void* stream);
/* Reverse of ugks_wall_loads with respect to F: F_bar [nface][dim+2]
   (written; zero off the walls) from the cotangents face_loads_bar and
   side_loads_bar (layouts as above; either may be NULL = zero). */
int ugks_wall_loads_adjoint(ugks_ctx* ctx, const double* face_loads_bar, const double* side_loads_bar,
                            double* F_bar, void* stream);
/* Cotangents of the prescribed motion and wall temperatures from the
   per-face cotangents face_bar [nface][5] of the reverse-mode entry points
   below: U_bar [nblock][2] = sum over the block's faces of the face grid
   velocity and wall velocity entries (the rigid block velocity moves both),
   rtw_bar [nblock][4] = sum of the wall RT entries over each side's faces.
   Sums in a fixed order. */
int ugks_param_bars(ugks_ctx* ctx, const double* face_bar, double* U_bar, double* rtw_bar, void* stream);

/*
 * Newton-Euler (3-DOF) rigid motion of block `blk` (Sec. 3, Step 1: a body
 * moves by the Newton-Euler equations driven by the gas, or by a given
 * motion), loosely coupled: the force and moment on the body at level n are
 * the area integrals of the macro flux into the block's wall sides from the
 * face macro flux F (device [nface][dim+2]; e.g. ugks_last_flux after the
 * last inner iteration of step n), the moment about the block's moved
 * rotation centre (the centre of mass), plus the constant external load of
 * body (host [5]: mass, moment of inertia, Fx, Fy, Mz).  pose (host [6], in
 * and out: dx, dy, th, ux, uy, om, as ugks_set_poses takes them) advances
 * by dt: u' = u + dt F/m, om' = om + dt M/I, then the position and angle by
 * the trapezoidal rule of the old and new velocities (exact for constant
 * loads).  The caller installs the new poses with ugks_set_poses.  Waits for
 * `stream`.  UGKS_E_UNSUPPORTED in 1D; UGKS_E_ARG for a bad block, a
 * non-positive mass, inertia or dt.
 */
int ugks_newton_euler(ugks_ctx* ctx, int32_t blk, const double* body, double dt, const double* F, double* pose,
                      void* stream);

/* Thread-local message of the last failure ("" if none). */
const char* ugks_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
