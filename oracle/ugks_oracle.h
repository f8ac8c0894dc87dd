/*
 * Plain FP64 CPU oracle of the implicit unsteady unified gas-kinetic scheme
 * (UGKS) on moving overset structured meshes.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link or
 * call this code; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code with the HIP library.
 *
 * Every routine follows the paper (Zhang, Long, Cao, Xu, "Unified Gas-Kinetic
 * Scheme for Unsteady Multiscale Flows with Moving Boundaries") step by step:
 *   Sec. 2.1  kinetic model, reduced distributions h and b, Shakhov equilibrium,
 *             finite-volume update, UGKS interface solution (Eq. fullSolution),
 *             ghost-cell and isothermal-wall boundaries (Eq. maxWalldes),
 *   Sec. 2.2  dual time stepping (Eqs. dualTimeStepping_macro/_micro,
 *             residual_macro_n, residual_micro_n+1,s), LU-SGS, Steps 1-8,
 *   Sec. 3    overset assembly and inverse-distance interpolation.
 * Where the paper is silent the reading taken is written next to the code.
 */
#ifndef UGKS_ORACLE_H
#define UGKS_ORACLE_H
#include <stdint.h>

/* Scalar type of every value: double.  The tangent build (ugks_oracle_tl.cpp)
   compiles this same source as C++ with a forward-mode dual number instead,
   which carries one directional derivative beside each value. */
#ifdef OR_TANGENT
#include "or_dual.h"
#else
typedef double real;
#endif

#ifdef __cplusplus
extern "C" {
#endif

/* block side boundary kinds */
enum { OR_PERIODIC = 0, OR_FARFIELD = 1, OR_COPY = 2, OR_WALL = 3, OR_NONE = 4 };
/* cell kinds */
enum { OR_HOLE = 0, OR_FIELD = 1, OR_RECEPTOR = 2 };

typedef struct or_case or_case;

/*
 * Create a case.
 *   dim         1 or 2 (monatomic gas: N_xi = 3 - dim internal components).
 *   gas[4]      Pr, omega, mu_ref, rt_ref.  tau = mu_ref (RT/rt_ref)^omega / p;
 *               mu_ref <= 0 means collisionless (1/tau = 0).
 *   nv[2]       nvx, nvy (nvy = 1 in 1D).
 *   vrange[4]   vx_min, vx_max, vy_min, vy_max of the uniform velocity grid.
 *   vx, vy      the velocity points (length nvx, nvy).
 *   winf[4]     far-field conservative state (rho, rho u, [rho v,] rho E).
 *   cfl[2]      CFL of the explicit flux time step and of the virtual step.
 *   nblock      number of structured blocks.
 *   bint        per block 6 ints: ni, nj, bc[i-min,i-max,j-min,j-max].
 *   bdbl        per block 14 doubles: rtw[4], vwx[4], vwy[4], xc0, yc0
 *               (wall RT and wall velocity added to the mesh velocity per
 *               side; reference rotation centre).
 *   nodes       per block the reference node coordinates: x then y, each
 *               (ni+1)*(nj+1) values, index i + (ni+1)*j (1D: x only, ni+1).
 * Returns NULL on bad input.
 */
or_case* or_create(int dim, const real* gas, const int* nv, const real* vrange,
                   const real* vx, const real* vy, const real* winf,
                   const real* cfl, int nblock, const int* bint,
                   const real* bdbl, const real* nodes);
void or_free(or_case* c);

int or_ncell(const or_case* c);
int or_nface(const or_case* c);
int or_nv(const or_case* c);

/* rigid pose of a block: translation (dx,dy), rotation th about the moved
   centre, and the rigid velocity (ux,uy) and angular velocity om. */
void or_set_pose(or_case* c, int blk, real dx, real dy, real th,
                 real ux, real uy, real om);
/* wall RT of side `side` (0 i-min, 1 i-max, 2 j-min, 3 j-max) of a wall
   block side, for the faces already built */
void or_set_wall_rt(or_case* c, int blk, int side, real rtw);
/* far-field conservative state (nw entries) and its Maxwellian, the value
   of far-field ghosts from the next step on */
void or_set_farfield(or_case* c, const real* winf);
/* node positions, cell and face geometry, face grid velocity at the current
   poses. */
void or_update_geometry(or_case* c);

/* replaces the uniform velocity grid by nv points (vx, vy) with cell
   volumes wk > 0 (an unstructured velocity mesh, 2D); call right after
   or_create.  0, or -1 on bad input (nothing changed). */
int or_set_dvs(or_case* c, int nv, const real* vx, const real* vy, const real* wk);
/* velocity points and quadrature weights V_k (k = ix + nvx*iy) */
void or_dvs(const or_case* c, real* vx, real* vy, real* wk);
/* one-axis composite Newton-Cotes weights (reading of the velocity grid) */
void or_nc_weights(int n, real a, real b, real* w);

/* geometry export: cell centroid [ncell][2], volume, metric [ncell][4];
   face L,R (cell or -1-side), normal [2], area, centre [2], grid velocity [2] */
void or_geometry(const or_case* c, real* cx, real* vol, real* g,
                 int* fl, int* fr, real* fn, real* fs, real* fx, real* fu);

/* structured position of every face: block, direction (0 i, 1 j) and the
   (i, j) of the face in its block's face grid */
void or_face_ids(const or_case* c, int* blk, int* dir, int* fi, int* fj);

void or_set_types(or_case* c, const int8_t* type);
void or_get_types(const or_case* c, int8_t* type);
void or_set_overset(or_case* c, int nrec, const int* rec, const int* ptr,
                    const int* don, const real* w);

/* discrete reduced Maxwellian (H,B) of W at every cell (no Shakhov part) */
void or_maxwellian(const or_case* c, const real* W, real* h, real* b);
/* W = sum_k V_k Psi_k f and q about the velocity of that W, every cell */
void or_moments(const or_case* c, const real* h, const real* b, real* W, real* q);
/* heat flux of f about the velocity of a given W (every cell) */
void or_heatflux(const or_case* c, const real* h, const real* b, const real* W, real* q);

/* explicit flux time step dt_s (global) and virtual steps dtp[ncell] */
real or_timesteps(const or_case* c, real* dtp);

/* time-integration coefficients q1..q5 of the interface solution */
void or_time_coeffs(real dts, real tau, real* q);
/* equilibrium slope and time coefficients: a[d][nw], A[nw] */
void or_slope_coeffs(int dim, real rho, const real* u, real lam,
                     const real* uf, const real* dW, real* a, real* A);
/* reduced Shakhov equilibrium at one velocity */
void or_shakhov(int dim, real pr, real rho, const real* u, real lam,
                const real* q, const real* v, real* hp, real* bp);

/* Step 1 / Step 3 flux: divergence D[ncell][nv] (h,b), face macro flux
   F[nface][nw] along the face normal, wall output [nface][1+nw]
   (rho_w, then the macro flux into the wall). */
void or_flux(const or_case* c, real dts, const real* h, const real* b,
             const real* W, const real* q, real* Dh, real* Db,
             real* F, real* wall);

/* wall loads from a face macro flux F [nface][nw]: face_out [nface][dim+3]
   (per wall face and unit area: momentum flux into the wall, its pressure
   and shear components, energy flux; zero elsewhere), side_out
   [nblock][4][4] (per block side: force x, y, its moment about the block's
   moved rotation centre, energy flux); either may be NULL */
void or_wall_loads(const or_case* c, const real* F, real* face_out, real* side_out);

/* Newton-Euler (3-DOF) step of block b's rigid motion driven by its wall
   loads from F [nface][nw] plus a constant external load:
   body = {mass, moment of inertia, Fx_ext, Fy_ext, M_ext}; pose [6] =
   {dx, dy, th, ux, uy, om} advanced by dt in place */
void or_newton_euler(const or_case* c, int b, const real* body, real dt, const real* F, real* pose);

/* overset interpolation of f, W, q into receptors */
void or_interp(const or_case* c, real* h, real* b, real* W, real* q);

/* Steps 1-2: source S = f^n/dt + r^n/2 and the level-n face flux Fn */
void or_begin_step(or_case* c, real dt, real dts, real* h, real* b,
                   real* W, real* q, real* Sh, real* Sb, real* Fn);
/* Steps 1-2 at listed cells only (same interpolation over the whole field):
   Sh, Sb [ns][nv] and the macro flux of each face slot of each listed cell,
   Fc [ns][4][nw] (zero where a slot has no face) */
void or_begin_step_cells(or_case* c, real dt, real dts, real* h, real* b, real* W, real* q,
                         int ns, const int* cells, real* Sh, real* Sb, real* Fc);
/* Steps 3-7, one inner iteration; resid[nw] = L2 norm of R over field cells;
   Fout[nface][nw] (may be NULL) receives the face macro flux of Step 3 */
void or_pseudo_step(const or_case* c, real dt, real dts, const real* dtp,
                    real* h, real* b, real* W, const real* Wn, real* q,
                    const real* Sh, const real* Sb, const real* Fn,
                    real* resid, real* Fout);

/* exposed pieces of one inner iteration, for tests */
void or_macro_lusgs(const or_case* c, real dt, const real* dtp, const real* W,
                    const real* Wn, const real* F, const real* Fn, real* Wp,
                    real* resid);
void or_micro_lusgs(const or_case* c, real dt, const real* dtp, const real* Wp,
                    const real* qp, real* h, real* b, const real* Sh,
                    const real* Sb, const real* Dh, const real* Db);
void or_step7(const or_case* c, const real* Wp, const real* h, const real* b, real* W);

/* overset assembly (hole cutting, buffer layer, donors and weights) at the
   current geometry.  wrule 0 = inverse distance squared, 1 = bilinear.
   overlap = fringe depth (cell layers) kept beside an overset boundary.
   Returns 0, or -5 if a receptor has no donor. */
int or_assemble(or_case* c, int wrule, int overlap, int* nrec_out);
int or_get_overset(const or_case* c, int* rec, int* ptr, int* don, real* w);
int or_overset_count(const or_case* c);
/* rows after the receptors: cells uncovered from holes, filled by the next or_begin_step */
int or_refill_count(const or_case* c);
/* current node coordinates, blocks concatenated, (ni+1)(nj+1) per block */
void or_nodes(const or_case* c, real* x, real* y);

#ifdef __cplusplus
}
#endif
#endif
