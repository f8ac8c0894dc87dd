/*
 * Plain FP64 CPU oracle of the implicit unsteady UGKS on moving overset
 * meshes.  TEST INFRASTRUCTURE ONLY (see ugks_oracle.h).
 *
 * Written for a reader holding the paper: every function names the passage it
 * follows.  No blocking, fusion or reordering beyond what the paper's steps
 * state; OpenMP only over independent velocities or over cells / faces that
 * write only their own results, so the results do not depend on the thread
 * count.  Build with -O2 -ffp-contract=off (no fused multiply-add).
 */
#include "ugks_oracle.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define PI 3.14159265358979323846

/* ------------------------------------------------------------------------ */
/* case data                                                                 */
/* ------------------------------------------------------------------------ */
typedef struct {
  int ni, nj, bc[4];
  real rtw[4], vwx[4], vwy[4], xc0, yc0;
  real *x0, *y0;          /* reference nodes */
  real dx, dy, th, ux, uy, om;
  int cell0;
} blk_t;

/* neighbour reference */
enum { NB_CELL = 0, NB_FF = 1, NB_COPY = 2, NB_WALL = 3, NB_MISSING = 4 };
typedef struct { int kind, cell; } nbref;

/* face kinds */
enum { F_INTERIOR = 0, F_GHOST = 1, F_WALL = 2 };

typedef struct {
  int kind;          /* F_INTERIOR: L and R are cells; F_GHOST: one side virtual;
                        F_WALL: one side is a wall */
  int L, R;          /* cells, or -1 for the virtual / wall side */
  int gkind, gcell;  /* ghost side: NB_FF or NB_COPY (gcell = copied cell) */
  int blk, side;     /* boundary side id for ghost / wall faces */
  int dir;           /* 0: i-face, 1: j-face */
  real nx, ny, S, xf, yf, ux, uy;
  real rtw, vwx, vwy;  /* wall temperature and wall velocity (lab frame) */
} face_t;

struct or_case {
  int dim, nxi, nw;
  real pr, omega, mu_ref, rt_ref, cfl_s, cfl_p;
  int nvx, nvy, nv;
  real vx0, vx1, vy0, vy1;
  real *vk_x, *vk_y, *wk;  /* per k */
  real winf[4];
  real *finf_h, *finf_b;   /* far-field Maxwellian per k */
  int nblock; blk_t* blk;
  int ncell;
  int8_t* type;
  int* cblk; int* ci; int* cj;
  real *xn, *yn;           /* current nodes, per block concatenated */
  int* node0;
  real *cx, *cy, *vol, *g; /* g: J^{-T}, 4 per cell */
  real* cdx;               /* [ncell][4][2] face centre (cell's own nodes) - centroid */
  int nface; face_t* face;
  int* cface;                /* [ncell][4] face ids (-1 none): i-low, i-high, j-low, j-high */
  int* csign;                /* [ncell][4] +1 if the face normal points out of the cell */
  int nrec; int *rec, *dptr, *don; real* dw;
  int nref;                  /* refill entries appended after the receptors */
};

int or_ncell(const or_case* c) { return c->ncell; }
int or_nface(const or_case* c) { return c->nface; }
int or_nv(const or_case* c) { return c->nv; }

/* ------------------------------------------------------------------------ */
/* velocity grid quadrature                                                  */
/* ------------------------------------------------------------------------ */
/*
 * Velocity-space weights V_k (Eq. macroscopicFlux).  The paper leaves the
 * rule for a uniform grid open; the reading taken (composite closed
 * Newton-Cotes on n uniform points):
 *   (n-1) % 4 == 0 : composite Boole
 *   n odd          : composite Simpson
 *   n % 4 == 0     : Simpson | 3/8 | Simpson with the 3/8 panel centred
 *   n % 4 == 2     : Simpson | 3/8 | 3/8 | 3/8 | Simpson, mirror symmetric
 *                    (n >= 10; n = 6: Simpson on 2 intervals, 3/8 on 3)
 *   n == 1 : weight 1;  n == 2 : trapezoid.
 * Every rule but n = 6 is mirror symmetric, so a resting Maxwellian keeps
 * zero odd moments.
 */
static void add_simpson(real* w, int i0, int m, real h) {
  for (int p = 0; p < m; p += 2) {
    w[i0 + p] += h / 3.0;
    w[i0 + p + 1] += 4.0 * h / 3.0;
    w[i0 + p + 2] += h / 3.0;
  }
}
static void add_38(real* w, int i0, real h) {
  w[i0] += 3.0 * h / 8.0;
  w[i0 + 1] += 9.0 * h / 8.0;
  w[i0 + 2] += 9.0 * h / 8.0;
  w[i0 + 3] += 3.0 * h / 8.0;
}
void or_nc_weights(int n, real a, real b, real* w) {
  for (int i = 0; i < n; i++) w[i] = 0.0;
  if (n == 1) { w[0] = 1.0; return; }
  real h = (b - a) / (n - 1);
  int m = n - 1;
  if (n == 2) { w[0] = w[1] = h / 2.0; return; }
  if (m % 4 == 0) {
    for (int p = 0; p < m; p += 4) {
      w[p] += 14.0 * h / 45.0;
      w[p + 1] += 64.0 * h / 45.0;
      w[p + 2] += 24.0 * h / 45.0;
      w[p + 3] += 64.0 * h / 45.0;
      w[p + 4] += 14.0 * h / 45.0;
    }
  } else if (n % 2 == 1) {
    add_simpson(w, 0, m, h);
  } else if (n % 4 == 0) {
    int m1 = (n - 4) / 2;
    add_simpson(w, 0, m1, h);
    add_38(w, m1, h);
    add_simpson(w, m1 + 3, m1, h);
  } else if (n >= 10) {
    int ms = (n - 4) / 2, m1 = ms - 3;
    add_simpson(w, 0, m1, h);
    add_38(w, m1, h);
    add_38(w, m1 + 3, h);
    add_38(w, m1 + 6, h);
    add_simpson(w, m1 + 9, m1, h);
  } else {
    add_simpson(w, 0, n - 4, h);
    add_38(w, n - 4, h);
  }
}

/* ------------------------------------------------------------------------ */
/* kinetic model, Sec. 2.1                                                   */
/* ------------------------------------------------------------------------ */
/* lambda = 1/(2RT) from W: rho E = rho|U|^2/2 + (D+N_xi) rho/(4 lambda) */
static void prim(const or_case* c, const real* W, real* rho, real* u, real* lam) {
  int d = c->dim;
  *rho = W[0];
  real ke = 0.0;
  for (int i = 0; i < d; i++) { u[i] = W[1 + i] / W[0]; ke += u[i] * u[i]; }
  for (int i = d; i < 2; i++) u[i] = 0.0;
  real e = W[d + 1] - 0.5 * W[0] * ke;
  *lam = (real)(d + c->nxi) * W[0] / (4.0 * e);
}

/* positive density and internal energy */
static int physical(const or_case* c, const real* W) {
  int d = c->dim;
  if (!(W[0] > 0.0)) return 0;
  real ke = 0.0;
  for (int i = 0; i < d; i++) ke += W[1 + i] * W[1 + i];
  real e = W[d + 1] - 0.5 * ke / W[0];
  return e > 0.0;
}

/* collision time tau = mu/p, mu = mu_ref (RT/RT_ref)^omega; 1/tau returned */
static real inv_tau(const or_case* c, real rho, real lam) {
  if (c->mu_ref <= 0.0) return 0.0;
  real rt = 1.0 / (2.0 * lam);
  real mu = c->mu_ref * pow(rt / c->rt_ref, c->omega);
  real p = rho * rt;
  return p / mu;
}

/* reduced Maxwellian H = rho (lam/pi)^{D/2} exp(-lam |v-U|^2), B = N_xi/(2 lam) H */
static void maxw(const or_case* c, real rho, const real* u, real lam,
                 real vx, real vy, real* H, real* B) {
  real cx = vx - u[0], cy = (c->dim == 2) ? vy - u[1] : 0.0;
  real nrm = rho * pow(lam / PI, 0.5 * c->dim);
  real e = nrm * exp(-lam * (cx * cx + cy * cy));
  *H = e;
  *B = (real)c->nxi / (2.0 * lam) * e;
}

/*
 * Reduced Shakhov correction (Sec. 2.1, H^+ and B^+), monatomic K = 0, with
 * the peculiar velocity c = v - U (the gas velocity):
 *   H+ = 4(1-Pr) lam^2/(5 rho) (c.q) (2 lam c^2 - 2 - D) H
 *   B+ = 4(1-Pr) lam^2/(5 rho) (c.q) (2 lam c^2 - D) N_xi H/(2 lam)
 */
void or_shakhov(int dim, real pr, real rho, const real* u, real lam,
                const real* q, const real* v, real* hp, real* bp) {
  int nxi = 3 - dim;
  real cx = v[0] - u[0], cy = (dim == 2) ? v[1] - u[1] : 0.0;
  real c2 = cx * cx + cy * cy;
  real cq = cx * q[0] + ((dim == 2) ? cy * q[1] : 0.0);
  real H = rho * pow(lam / PI, 0.5 * dim) * exp(-lam * c2);
  real s = 4.0 * (1.0 - pr) * lam * lam / (5.0 * rho) * cq;
  *hp = s * (2.0 * lam * c2 - 2.0 - dim) * H;
  *bp = s * (2.0 * lam * c2 - dim) * (real)nxi * H / (2.0 * lam);
}

/* ------------------------------------------------------------------------ */
/* Gaussian moments and the slope / time-derivative coefficients             */
/* (Sec. 2.1: f+ ~ g0 + g0+ + x.grad g0 + t dg0/dt; grad g0 = g0 (a.psi),     */
/*  dg0/dt = g0 (A.psi), with psi = (1, v, (v^2 + xi^2)/2))                   */
/* ------------------------------------------------------------------------ */
typedef struct { int n; real c[8]; int px[8], py[8], r[8]; } poly;

static poly psi_poly(int dim, int a) {
  poly p; p.n = 0;
  if (a == 0) { p.n = 1; p.c[0] = 1; p.px[0] = 0; p.py[0] = 0; p.r[0] = 0; return p; }
  if (a <= dim) {
    p.n = 1; p.c[0] = 1; p.px[0] = (a == 1); p.py[0] = (a == 2); p.r[0] = 0; return p;
  }
  /* energy: (vx^2 + vy^2 + xi^2)/2 */
  p.c[p.n] = 0.5; p.px[p.n] = 2; p.py[p.n] = 0; p.r[p.n] = 0; p.n++;
  if (dim == 2) { p.c[p.n] = 0.5; p.px[p.n] = 0; p.py[p.n] = 2; p.r[p.n] = 0; p.n++; }
  p.c[p.n] = 0.5; p.px[p.n] = 0; p.py[p.n] = 0; p.r[p.n] = 1; p.n++;
  return p;
}

/* <psi_a * v_dir^e * psi_b> under the normalised Maxwellian (rho = 1) */
static real gmom(int dim, const real* mx, const real* my, const real* mxi,
                   int a, int b, int dir, int e) {
  poly pa = psi_poly(dim, a), pb = psi_poly(dim, b);
  real s = 0.0;
  for (int i = 0; i < pa.n; i++)
    for (int j = 0; j < pb.n; j++) {
      int px = pa.px[i] + pb.px[j] + ((dir == 0) ? e : 0);
      int py = pa.py[i] + pb.py[j] + ((dir == 1) ? e : 0);
      int r = pa.r[i] + pb.r[j];
      s += pa.c[i] * pb.c[j] * mx[px] * my[py] * mxi[r];
    }
  return s;
}

/* raw moments of a 1D Gaussian with mean u and variance 1/(2 lam) */
static void gauss1(real u, real lam, int nmax, real* m) {
  m[0] = 1.0;
  m[1] = u;
  for (int n = 1; n < nmax; n++) m[n + 1] = u * m[n] + (real)n / (2.0 * lam) * m[n - 1];
}

/* plain Gaussian elimination with partial pivoting, n <= 4 */
static void solve(int n, real* M, real* x) {
  for (int k = 0; k < n; k++) {
    int p = k;
    for (int i = k + 1; i < n; i++)
      if (fabs(M[i * n + k]) > fabs(M[p * n + k])) p = i;
    if (p != k) {
      for (int j = 0; j < n; j++) { real t = M[k * n + j]; M[k * n + j] = M[p * n + j]; M[p * n + j] = t; }
      real t = x[k]; x[k] = x[p]; x[p] = t;
    }
    for (int i = k + 1; i < n; i++) {
      real f = M[i * n + k] / M[k * n + k];
      for (int j = k; j < n; j++) M[i * n + j] -= f * M[k * n + j];
      x[i] -= f * x[k];
    }
  }
  for (int i = n - 1; i >= 0; i--) {
    real s = x[i];
    for (int j = i + 1; j < n; j++) s -= M[i * n + j] * x[j];
    x[i] = s / M[i * n + i];
  }
}

/*
 * a_d solves <psi psi^T> a_d = (dW/dx_d)/rho (the moments of grad g0 equal the
 * gradient of the conservative variables), and A solves the compatibility
 * condition <psi (A.psi + sum_d w_d a_d.psi)> = 0 with the relative velocity
 * w = v - U_f of the moving face (Eq. BGK: w = v - U).  Moments are the
 * analytic Gaussian ones.  dW is [dim][nw], a is [dim][nw].
 */
void or_slope_coeffs(int dim, real rho, const real* u, real lam,
                     const real* uf, const real* dW, real* a, real* A) {
  int nw = dim + 2, nxi = 3 - dim;
  real mx[8], my[8], mxi[3];
  gauss1(u[0], lam, 7, mx);
  if (dim == 2) gauss1(u[1], lam, 7, my);
  else { for (int i = 0; i < 8; i++) my[i] = (i == 0) ? 1.0 : 0.0; }
  mxi[0] = 1.0;
  mxi[1] = (real)nxi / (2.0 * lam);
  mxi[2] = (real)nxi * (nxi + 2) / (4.0 * lam * lam);
  real M[16], Mc[16], rhs[4];
  for (int i = 0; i < nw; i++)
    for (int j = 0; j < nw; j++) M[i * nw + j] = gmom(dim, mx, my, mxi, i, j, 0, 0);
  real b[4] = {0, 0, 0, 0};
  for (int d = 0; d < dim; d++) {
    memcpy(Mc, M, sizeof(real) * nw * nw);
    for (int i = 0; i < nw; i++) rhs[i] = dW[d * nw + i] / rho;
    solve(nw, Mc, rhs);
    for (int i = 0; i < nw; i++) a[d * nw + i] = rhs[i];
    /* b -= <psi w_d (a_d.psi)> with w_d = v_d - uf_d */
    for (int i = 0; i < nw; i++) {
      real s = 0.0;
      for (int j = 0; j < nw; j++)
        s += (gmom(dim, mx, my, mxi, i, j, d, 1) - uf[d] * M[i * nw + j]) * a[d * nw + j];
      b[i] -= s;
    }
  }
  memcpy(Mc, M, sizeof(real) * nw * nw);
  solve(nw, Mc, b);
  for (int i = 0; i < nw; i++) A[i] = b[i];
}

/* (a.psi) integrated over xi, for h (m = 0) and for b (m = 1):
   a0 + a.v + a_E/2 (|v|^2 + (N_xi + 2m)/(2 lam)) */
static real apsi(int dim, const real* a, real vx, real vy, real lam, int m) {
  int nxi = 3 - dim;
  real v2 = vx * vx + ((dim == 2) ? vy * vy : 0.0);
  real s = a[0] + a[1] * vx;
  if (dim == 2) s += a[2] * vy;
  s += 0.5 * a[dim + 1] * (v2 + (real)(nxi + 2 * m) / (2.0 * lam));
  return s;
}

/*
 * Time integrals over [0, dts] of c1..c5 (Eq. fullSolution):
 *   q1 = tau(1-e), q2 = tau^2(-1+(1+x)e), q3 = dts - q1,
 *   q4 = tau^2(2-x-(2+x)e), q5 = tau^2(x^2/2 - x + 1 - e),  x = dts/tau, e = exp(-x).
 * For x < 1 the same integrals are summed as their Taylor series (m <= 24),
 * which keeps every digit as tau grows (the closed forms cancel like 1/x^3);
 * tau = inf is x = 0.
 */
void or_time_coeffs(real dts, real tau, real* q) {
  real x = isinf(tau) ? 0.0 : dts / tau;
  if (x < 1.0) {
    real s1 = 0, s2 = 0, s3 = 0, s4 = 0, s5 = 0;
    real fact = 1.0, xp = 1.0; /* xp = x^(m-1) at the top of step m */
    real xpm2 = 0.0;
    for (int m = 1; m <= 24; m++) {
      fact *= m;
      real sg = (m % 2 == 0) ? 1.0 : -1.0; /* (-1)^m */
      s1 += -sg * xp / fact;
      if (m >= 2) {
        s3 += sg * xp / fact;
        s2 += -sg * (m - 1) * xpm2 / fact;
      }
      if (m >= 3) {
        s4 += sg * (m - 2) * xpm2 / fact;
        s5 += -sg * xpm2 / fact;
      }
      xpm2 = (m == 1) ? 1.0 : xpm2 * x;
      xp *= x;
    }
    q[0] = dts * s1;
    q[1] = dts * dts * s2;
    q[2] = dts * s3;
    q[3] = dts * dts * s4;
    q[4] = dts * dts * s5;
  } else {
    real e = exp(-x);
    q[0] = tau * (1.0 - e);
    q[1] = tau * tau * (-1.0 + (1.0 + x) * e);
    q[2] = dts - q[0];
    q[3] = tau * tau * (2.0 - x - (2.0 + x) * e);
    q[4] = tau * tau * (0.5 * x * x - x + 1.0 - e);
  }
}

/* ------------------------------------------------------------------------ */
/* mesh                                                                      */
/* ------------------------------------------------------------------------ */
static int cell_index(const or_case* c, int b, int i, int j) {
  return c->blk[b].cell0 + i + c->blk[b].ni * j;
}

/* neighbour of cell (b,i,j) one step along dir (0: i, 1: j), side -1 / +1 */
static nbref nbr(const or_case* c, int cell, int dir, int side) {
  nbref r = {NB_MISSING, -1};
  int b = c->cblk[cell], i = c->ci[cell], j = c->cj[cell];
  const blk_t* B = &c->blk[b];
  int ii = i + ((dir == 0) ? side : 0), jj = j + ((dir == 1) ? side : 0);
  int sid = -1;
  if (dir == 0 && (ii < 0 || ii >= B->ni)) {
    if (B->bc[0] == OR_PERIODIC) ii = (ii + B->ni) % B->ni;
    else sid = (ii < 0) ? 0 : 1;
  }
  if (dir == 1 && (jj < 0 || jj >= B->nj)) {
    if (B->bc[2] == OR_PERIODIC) jj = (jj + B->nj) % B->nj;
    else sid = (jj < 0) ? 2 : 3;
  }
  if (sid < 0) {
    int n = cell_index(c, b, ii, jj);
    if (c->type[n] == OR_HOLE) return r;
    r.kind = NB_CELL; r.cell = n; return r;
  }
  switch (B->bc[sid]) {
    case OR_FARFIELD: r.kind = NB_FF; break;
    case OR_COPY: r.kind = NB_COPY; r.cell = cell; break;
    case OR_WALL: r.kind = NB_WALL; break;
    default: r.kind = NB_MISSING; break;
  }
  return r;
}

static void build_faces(or_case* c) {
  int cap = 0;
  for (int b = 0; b < c->nblock; b++) {
    const blk_t* B = &c->blk[b];
    cap += (B->ni + 1) * B->nj + ((c->dim == 2) ? B->ni * (B->nj + 1) : 0);
  }
  c->face = (face_t*)calloc(cap > 0 ? cap : 1, sizeof(face_t));
  c->cface = (int*)malloc(sizeof(int) * 4 * c->ncell);
  c->csign = (int*)malloc(sizeof(int) * 4 * c->ncell);
  for (int i = 0; i < 4 * c->ncell; i++) { c->cface[i] = -1; c->csign[i] = 0; }
  int nf = 0;
  for (int b = 0; b < c->nblock; b++) {
    blk_t* B = &c->blk[b];
    for (int dir = 0; dir < c->dim; dir++) {
      int per = (B->bc[2 * dir] == OR_PERIODIC);
      int nI = (dir == 0) ? B->ni + 1 : B->ni;
      int nJ = (dir == 0) ? B->nj : B->nj + 1;
      for (int j = 0; j < nJ; j++)
        for (int i = 0; i < nI; i++) {
          if (dir == 0 && per && i == B->ni) continue;
          if (dir == 1 && per && j == B->nj) continue;
          face_t F; memset(&F, 0, sizeof(F));
          F.blk = b; F.L = -1; F.R = -1; F.side = -1; F.dir = dir;
          int lo_side = (dir == 0) ? 0 : 2, hi_side = lo_side + 1;
          int n = (dir == 0) ? B->ni : B->nj;
          int idx = (dir == 0) ? i : j;
          if (idx > 0) F.L = cell_index(c, b, (dir == 0) ? i - 1 : i, (dir == 0) ? j : j - 1);
          else if (per) F.L = (dir == 0) ? cell_index(c, b, B->ni - 1, j) : cell_index(c, b, i, B->nj - 1);
          if (idx < n) F.R = cell_index(c, b, i, j);
          int sid = -1;
          if (F.L < 0) sid = lo_side;
          if (F.R < 0) sid = hi_side;
          if (sid >= 0) {
            int bc = B->bc[sid];
            if (bc == OR_NONE || bc == OR_PERIODIC) continue;
            F.side = sid;
            if (bc == OR_WALL) {
              F.kind = F_WALL;
              F.rtw = B->rtw[sid];
            } else {
              F.kind = F_GHOST;
              int inner = (F.L >= 0) ? F.L : F.R;
              F.gkind = (bc == OR_FARFIELD) ? NB_FF : NB_COPY;
              F.gcell = inner;
            }
          } else F.kind = F_INTERIOR;
          c->face[nf] = F;
          if (F.L >= 0) {
            int slot = 2 * dir + 1;
            c->cface[4 * F.L + slot] = nf; c->csign[4 * F.L + slot] = +1;
          }
          if (F.R >= 0) {
            int slot = 2 * dir;
            c->cface[4 * F.R + slot] = nf; c->csign[4 * F.R + slot] = -1;
          }
          nf++;
        }
    }
  }
  c->nface = nf;
}

static real node_x(const or_case* c, int b, int i, int j) {
  return c->xn[c->node0[b] + i + (c->blk[b].ni + 1) * j];
}
static real node_y(const or_case* c, int b, int i, int j) {
  return c->yn[c->node0[b] + i + (c->blk[b].ni + 1) * j];
}

void or_set_pose(or_case* c, int b, real dx, real dy, real th, real ux,
                 real uy, real om) {
  blk_t* B = &c->blk[b];
  B->dx = dx; B->dy = dy; B->th = th; B->ux = ux; B->uy = uy; B->om = om;
}

/* wall RT of one side of a block (the isothermal wall of Eq. maxWalldes) */
void or_set_wall_rt(or_case* c, int b, int side, real rtw) {
  c->blk[b].rtw[side] = rtw;
  for (int f = 0; f < c->nface; f++) {
    face_t* F = &c->face[f];
    if (F->kind == F_WALL && F->blk == b && F->side == side) F->rtw = rtw;
  }
}

/* far-field state W_inf and its Maxwellian (the ghost value of far-field
   sides, Sec. 2.1) */
void or_set_farfield(or_case* c, const real* winf) {
  for (int i = 0; i < c->nw; i++) c->winf[i] = winf[i];
  real rho, u[2], lam;
  prim(c, c->winf, &rho, u, &lam);
  for (int k = 0; k < c->nv; k++) maxw(c, rho, u, lam, c->vk_x[k], c->vk_y[k], &c->finf_h[k], &c->finf_b[k]);
}

/* rigid motion: x = xc0 + d + R(th)(x0 - xc0); U = u + om x (x - xc0 - d) */
void or_update_geometry(or_case* c) {
  for (int b = 0; b < c->nblock; b++) {
    blk_t* B = &c->blk[b];
    int nn = (B->ni + 1) * ((c->dim == 2) ? (B->nj + 1) : 1);
    real cs = cos(B->th), sn = sin(B->th);
    for (int n = 0; n < nn; n++) {
      real rx = B->x0[n] - B->xc0;
      real ry = (c->dim == 2) ? B->y0[n] - B->yc0 : 0.0;
      c->xn[c->node0[b] + n] = B->xc0 + B->dx + (cs * rx - sn * ry);
      c->yn[c->node0[b] + n] = (c->dim == 2) ? B->yc0 + B->dy + (sn * rx + cs * ry) : 0.0;
    }
  }
  /* cells */
  for (int n = 0; n < c->ncell; n++) {
    int b = c->cblk[n], i = c->ci[n], j = c->cj[n];
    if (c->dim == 1) {
      real xa = node_x(c, b, i, 0), xb = node_x(c, b, i + 1, 0);
      c->vol[n] = xb - xa;
      c->cx[n] = 0.5 * (xa + xb); c->cy[n] = 0.0;
      c->g[4 * n + 0] = 1.0 / (xb - xa);
      c->g[4 * n + 1] = c->g[4 * n + 2] = c->g[4 * n + 3] = 0.0;
      for (int q = 0; q < 8; q++) c->cdx[8 * n + q] = 0.0;
      c->cdx[8 * n + 0] = xa - c->cx[n];
      c->cdx[8 * n + 2] = xb - c->cx[n];
      continue;
    }
    real px[4] = {node_x(c, b, i, j), node_x(c, b, i + 1, j), node_x(c, b, i + 1, j + 1), node_x(c, b, i, j + 1)};
    real py[4] = {node_y(c, b, i, j), node_y(c, b, i + 1, j), node_y(c, b, i + 1, j + 1), node_y(c, b, i, j + 1)};
    real A = 0.0, sx = 0.0, sy = 0.0;
    for (int k = 0; k < 4; k++) {
      int k1 = (k + 1) % 4;
      real cr = px[k] * py[k1] - px[k1] * py[k];
      A += cr; sx += (px[k] + px[k1]) * cr; sy += (py[k] + py[k1]) * cr;
    }
    A *= 0.5;
    c->vol[n] = A;
    c->cx[n] = sx / (6.0 * A);
    c->cy[n] = sy / (6.0 * A);
    /* metric from face-centre differences: J = [[x_xi, x_eta],[y_xi, y_eta]] */
    real xxi = 0.5 * (px[1] + px[2]) - 0.5 * (px[0] + px[3]);
    real yxi = 0.5 * (py[1] + py[2]) - 0.5 * (py[0] + py[3]);
    real xet = 0.5 * (px[3] + px[2]) - 0.5 * (px[0] + px[1]);
    real yet = 0.5 * (py[3] + py[2]) - 0.5 * (py[0] + py[1]);
    real det = xxi * yet - xet * yxi;
    /* grad f = J^{-T} (df/dxi, df/deta) */
    c->g[4 * n + 0] = yet / det;
    c->g[4 * n + 1] = -yxi / det;
    c->g[4 * n + 2] = -xet / det;
    c->g[4 * n + 3] = xxi / det;
    /* face centres from the cell's own nodes: i-low, i-high, j-low, j-high */
    real fxs[4] = {0.5 * (px[0] + px[3]), 0.5 * (px[1] + px[2]), 0.5 * (px[0] + px[1]), 0.5 * (px[3] + px[2])};
    real fys[4] = {0.5 * (py[0] + py[3]), 0.5 * (py[1] + py[2]), 0.5 * (py[0] + py[1]), 0.5 * (py[3] + py[2])};
    for (int q = 0; q < 4; q++) {
      c->cdx[8 * n + 2 * q] = fxs[q] - c->cx[n];
      c->cdx[8 * n + 2 * q + 1] = fys[q] - c->cy[n];
    }
  }
  /* faces */
  for (int f = 0; f < c->nface; f++) {
    face_t* F = &c->face[f];
    int b = F->blk;
    blk_t* B = &c->blk[b];
    int cell = (F->R >= 0) ? F->R : F->L;
    int i = c->ci[cell], j = c->cj[cell];
    /* recover the face's structured position from its adjacent cell */
    int dir = F->dir, fi, fj;
    if (F->R >= 0) { fi = c->ci[F->R]; fj = c->cj[F->R]; }
    else { fi = (dir == 0) ? i + 1 : i; fj = (dir == 1) ? j + 1 : j; }
    if (c->dim == 1) {
      F->S = 1.0; F->nx = 1.0; F->ny = 0.0;
      F->xf = node_x(c, b, fi, 0); F->yf = 0.0;
    } else {
      real x0, y0, x1, y1;
      if (dir == 0) {
        x0 = node_x(c, b, fi, fj); y0 = node_y(c, b, fi, fj);
        x1 = node_x(c, b, fi, fj + 1); y1 = node_y(c, b, fi, fj + 1);
      } else {
        x0 = node_x(c, b, fi, fj); y0 = node_y(c, b, fi, fj);
        x1 = node_x(c, b, fi + 1, fj); y1 = node_y(c, b, fi + 1, fj);
      }
      real ex = x1 - x0, ey = y1 - y0;
      F->S = sqrt(ex * ex + ey * ey);
      if (dir == 0) { F->nx = ey / F->S; F->ny = -ex / F->S; }
      else { F->nx = -ey / F->S; F->ny = ex / F->S; }
      F->xf = 0.5 * (x0 + x1); F->yf = 0.5 * (y0 + y1);
    }
    real rx = F->xf - (B->xc0 + B->dx), ry = F->yf - (B->yc0 + B->dy);
    F->ux = B->ux - B->om * ry;
    F->uy = (c->dim == 2) ? B->uy + B->om * rx : 0.0;
    if (F->kind == F_WALL) {
      F->vwx = F->ux + B->vwx[F->side];
      F->vwy = (c->dim == 2) ? F->uy + B->vwy[F->side] : 0.0;
    }
  }
}

or_case* or_create(int dim, const real* gas, const int* nv, const real* vrange,
                   const real* vx, const real* vy, const real* winf,
                   const real* cfl, int nblock, const int* bint,
                   const real* bdbl, const real* nodes) {
  if (dim != 1 && dim != 2) return NULL;
  or_case* c = (or_case*)calloc(1, sizeof(or_case));
  c->dim = dim; c->nxi = 3 - dim; c->nw = dim + 2;
  c->pr = gas[0]; c->omega = gas[1]; c->mu_ref = gas[2]; c->rt_ref = gas[3];
  c->cfl_s = cfl[0]; c->cfl_p = cfl[1];
  c->nvx = nv[0]; c->nvy = (dim == 2) ? nv[1] : 1; c->nv = c->nvx * c->nvy;
  c->vx0 = vrange[0]; c->vx1 = vrange[1]; c->vy0 = vrange[2]; c->vy1 = vrange[3];
  for (int i = 0; i < 4; i++) c->winf[i] = winf[i];
  real* wx = (real*)malloc(sizeof(real) * c->nvx);
  real* wy = (real*)malloc(sizeof(real) * c->nvy);
  or_nc_weights(c->nvx, c->vx0, c->vx1, wx);
  if (dim == 2) or_nc_weights(c->nvy, c->vy0, c->vy1, wy); else wy[0] = 1.0;
  c->vk_x = (real*)malloc(sizeof(real) * c->nv);
  c->vk_y = (real*)malloc(sizeof(real) * c->nv);
  c->wk = (real*)malloc(sizeof(real) * c->nv);
  for (int iy = 0; iy < c->nvy; iy++)
    for (int ix = 0; ix < c->nvx; ix++) {
      int k = ix + c->nvx * iy;
      c->vk_x[k] = vx[ix];
      c->vk_y[k] = (dim == 2) ? vy[iy] : 0.0;
      c->wk[k] = wx[ix] * wy[iy];
    }
  free(wx); free(wy);
  /* far-field Maxwellian */
  c->finf_h = (real*)malloc(sizeof(real) * c->nv);
  c->finf_b = (real*)malloc(sizeof(real) * c->nv);
  {
    real rho, u[2], lam;
    prim(c, c->winf, &rho, u, &lam);
    for (int k = 0; k < c->nv; k++) maxw(c, rho, u, lam, c->vk_x[k], c->vk_y[k], &c->finf_h[k], &c->finf_b[k]);
  }
  c->nblock = nblock;
  c->blk = (blk_t*)calloc(nblock, sizeof(blk_t));
  c->node0 = (int*)malloc(sizeof(int) * nblock);
  int ncell = 0, nnode = 0;
  const real* np = nodes;
  for (int b = 0; b < nblock; b++) {
    blk_t* B = &c->blk[b];
    B->ni = bint[6 * b]; B->nj = (dim == 2) ? bint[6 * b + 1] : 1;
    for (int s = 0; s < 4; s++) B->bc[s] = bint[6 * b + 2 + s];
    for (int s = 0; s < 4; s++) {
      B->rtw[s] = bdbl[14 * b + s];
      B->vwx[s] = bdbl[14 * b + 4 + s];
      B->vwy[s] = bdbl[14 * b + 8 + s];
    }
    B->xc0 = bdbl[14 * b + 12]; B->yc0 = bdbl[14 * b + 13];
    if ((B->bc[0] == OR_PERIODIC) != (B->bc[1] == OR_PERIODIC)) { or_free(c); return NULL; }
    if ((B->bc[2] == OR_PERIODIC) != (B->bc[3] == OR_PERIODIC)) { or_free(c); return NULL; }
    int nn = (B->ni + 1) * ((dim == 2) ? (B->nj + 1) : 1);
    B->x0 = (real*)malloc(sizeof(real) * nn);
    B->y0 = (real*)malloc(sizeof(real) * nn);
    memcpy(B->x0, np, sizeof(real) * nn); np += nn;
    if (dim == 2) { memcpy(B->y0, np, sizeof(real) * nn); np += nn; }
    else memset(B->y0, 0, sizeof(real) * nn);
    B->cell0 = ncell;
    c->node0[b] = nnode;
    ncell += B->ni * B->nj;
    nnode += nn;
  }
  c->ncell = ncell;
  c->type = (int8_t*)malloc(ncell);
  memset(c->type, OR_FIELD, ncell);
  c->cblk = (int*)malloc(sizeof(int) * ncell);
  c->ci = (int*)malloc(sizeof(int) * ncell);
  c->cj = (int*)malloc(sizeof(int) * ncell);
  for (int b = 0; b < nblock; b++)
    for (int j = 0; j < c->blk[b].nj; j++)
      for (int i = 0; i < c->blk[b].ni; i++) {
        int n = cell_index(c, b, i, j);
        c->cblk[n] = b; c->ci[n] = i; c->cj[n] = j;
      }
  c->xn = (real*)malloc(sizeof(real) * nnode);
  c->yn = (real*)malloc(sizeof(real) * nnode);
  c->cx = (real*)malloc(sizeof(real) * ncell);
  c->cy = (real*)malloc(sizeof(real) * ncell);
  c->vol = (real*)malloc(sizeof(real) * ncell);
  c->g = (real*)malloc(sizeof(real) * 4 * ncell);
  c->cdx = (real*)malloc(sizeof(real) * 8 * ncell);
  build_faces(c);
  or_update_geometry(c);
  return c;
}

void or_free(or_case* c) {
  if (!c) return;
  for (int b = 0; b < c->nblock; b++) { free(c->blk[b].x0); free(c->blk[b].y0); }
  free(c->blk); free(c->node0); free(c->vk_x); free(c->vk_y); free(c->wk);
  free(c->finf_h); free(c->finf_b); free(c->type); free(c->cblk); free(c->ci); free(c->cj);
  free(c->xn); free(c->yn); free(c->cx); free(c->cy); free(c->vol); free(c->g); free(c->cdx);
  free(c->face); free(c->cface); free(c->csign);
  free(c->rec); free(c->dptr); free(c->don); free(c->dw);
  free(c);
}

/* Unstructured discrete velocity space (Sec. 2.1: V_k is the volume of the
   k-th cell of the velocity mesh): the points and their cell areas replace
   the uniform grid; the far-field Maxwellian follows.  2D only. */
int or_set_dvs(or_case* c, int nv, const real* vx, const real* vy, const real* wk) {
  if (c->dim != 2 || nv < 1) return -1;
  for (int k = 0; k < nv; k++)
    if (!(wk[k] > 0.0)) return -1;
  free(c->vk_x); free(c->vk_y); free(c->wk); free(c->finf_h); free(c->finf_b);
  c->nv = nv; c->nvx = nv; c->nvy = 1;
  c->vk_x = (real*)malloc(sizeof(real) * nv);
  c->vk_y = (real*)malloc(sizeof(real) * nv);
  c->wk = (real*)malloc(sizeof(real) * nv);
  c->finf_h = (real*)malloc(sizeof(real) * nv);
  c->finf_b = (real*)malloc(sizeof(real) * nv);
  for (int k = 0; k < nv; k++) { c->vk_x[k] = vx[k]; c->vk_y[k] = vy[k]; c->wk[k] = wk[k]; }
  real rho, u[2], lam;
  prim(c, c->winf, &rho, u, &lam);
  for (int k = 0; k < nv; k++) maxw(c, rho, u, lam, c->vk_x[k], c->vk_y[k], &c->finf_h[k], &c->finf_b[k]);
  return 0;
}

void or_dvs(const or_case* c, real* vx, real* vy, real* wk) {
  for (int k = 0; k < c->nv; k++) { vx[k] = c->vk_x[k]; vy[k] = c->vk_y[k]; wk[k] = c->wk[k]; }
}

void or_geometry(const or_case* c, real* cx, real* vol, real* g, int* fl, int* fr,
                 real* fn, real* fs, real* fx, real* fu) {
  for (int n = 0; n < c->ncell; n++) {
    cx[2 * n] = c->cx[n]; cx[2 * n + 1] = c->cy[n]; vol[n] = c->vol[n];
    for (int i = 0; i < 4; i++) g[4 * n + i] = c->g[4 * n + i];
  }
  for (int f = 0; f < c->nface; f++) {
    const face_t* F = &c->face[f];
    fl[f] = (F->L >= 0) ? F->L : -1 - F->side;
    fr[f] = (F->R >= 0) ? F->R : -1 - F->side;
    fn[2 * f] = F->nx; fn[2 * f + 1] = F->ny; fs[f] = F->S;
    fx[2 * f] = F->xf; fx[2 * f + 1] = F->yf;
    fu[2 * f] = F->ux; fu[2 * f + 1] = F->uy;
  }
}

void or_nodes(const or_case* c, real* x, real* y) {
  int nn = 0;
  for (int b = 0; b < c->nblock; b++) nn += (c->blk[b].ni + 1) * (c->blk[b].nj + 1);
  memcpy(x, c->xn, sizeof(real) * nn);
  memcpy(y, c->yn, sizeof(real) * nn);
}

void or_face_ids(const or_case* c, int* blk, int* dir, int* fi, int* fj) {
  for (int f = 0; f < c->nface; f++) {
    const face_t* F = &c->face[f];
    blk[f] = F->blk;
    dir[f] = F->dir;
    if (F->R >= 0) { fi[f] = c->ci[F->R]; fj[f] = c->cj[F->R]; }
    else {
      fi[f] = c->ci[F->L] + (F->dir == 0 ? 1 : 0);
      fj[f] = c->cj[F->L] + (F->dir == 1 ? 1 : 0);
    }
  }
}

void or_set_types(or_case* c, const int8_t* type) { memcpy(c->type, type, c->ncell); }
void or_get_types(const or_case* c, int8_t* type) { memcpy(type, c->type, c->ncell); }

void or_set_overset(or_case* c, int nrec, const int* rec, const int* ptr, const int* don,
                    const real* w) {
  free(c->rec); free(c->dptr); free(c->don); free(c->dw);
  c->nrec = nrec;
  c->nref = 0;
  c->rec = (int*)malloc(sizeof(int) * (nrec > 0 ? nrec : 1));
  c->dptr = (int*)malloc(sizeof(int) * (nrec + 1));
  int nd = (nrec > 0) ? ptr[nrec] : 0;
  c->don = (int*)malloc(sizeof(int) * (nd > 0 ? nd : 1));
  c->dw = (real*)malloc(sizeof(real) * (nd > 0 ? nd : 1));
  if (nrec > 0) memcpy(c->rec, rec, sizeof(int) * nrec);
  memcpy(c->dptr, ptr, sizeof(int) * (nrec + 1));
  if (nd > 0) { memcpy(c->don, don, sizeof(int) * nd); memcpy(c->dw, w, sizeof(real) * nd); }
}

int or_overset_count(const or_case* c) { return c->nrec; }
int or_refill_count(const or_case* c) { return c->nref; }

int or_get_overset(const or_case* c, int* rec, int* ptr, int* don, real* w) {
  if (rec) memcpy(rec, c->rec, sizeof(int) * c->nrec);
  if (ptr) memcpy(ptr, c->dptr, sizeof(int) * (c->nrec + 1));
  int nd = c->dptr ? c->dptr[c->nrec] : 0;
  if (don && nd) memcpy(don, c->don, sizeof(int) * nd);
  if (w && nd) memcpy(w, c->dw, sizeof(real) * nd);
  return nd;
}

/* ------------------------------------------------------------------------ */
/* moments (Sec. 2.1: W = int Psi f, q = 1/2 int c (c^2 + xi^2) f)           */
/* ------------------------------------------------------------------------ */
static void cell_moments(const or_case* c, const real* h, const real* b, real* W) {
  int d = c->dim;
  for (int m = 0; m < c->nw; m++) W[m] = 0.0;
  for (int k = 0; k < c->nv; k++) {
    real vx = c->vk_x[k], vy = c->vk_y[k], w = c->wk[k];
    W[0] += w * h[k];
    W[1] += w * vx * h[k];
    if (d == 2) W[2] += w * vy * h[k];
    W[d + 1] += w * 0.5 * ((vx * vx + vy * vy) * h[k] + b[k]);
  }
}
static void cell_heatflux(const or_case* c, const real* h, const real* b,
                          const real* u, real* q) {
  q[0] = q[1] = 0.0;
  for (int k = 0; k < c->nv; k++) {
    real cx = c->vk_x[k] - u[0], cy = (c->dim == 2) ? c->vk_y[k] - u[1] : 0.0;
    real e = (cx * cx + cy * cy) * h[k] + b[k];
    q[0] += c->wk[k] * 0.5 * cx * e;
    if (c->dim == 2) q[1] += c->wk[k] * 0.5 * cy * e;
  }
}

void or_moments(const or_case* c, const real* h, const real* b, real* W, real* q) {
#pragma omp parallel for schedule(static)
  for (int n = 0; n < c->ncell; n++) {
    const real* hn = h + (size_t)n * c->nv;
    const real* bn = b + (size_t)n * c->nv;
    cell_moments(c, hn, bn, W + (size_t)n * c->nw);
    real rho, u[2], lam;
    prim(c, W + (size_t)n * c->nw, &rho, u, &lam);
    if (q) {
      real qq[2];
      cell_heatflux(c, hn, bn, u, qq);
      for (int i = 0; i < c->dim; i++) q[(size_t)n * c->dim + i] = qq[i];
    }
  }
}

void or_heatflux(const or_case* c, const real* h, const real* b, const real* W, real* q) {
#pragma omp parallel for schedule(static)
  for (int n = 0; n < c->ncell; n++) {
    real rho, u[2], lam;
    prim(c, W + (size_t)n * c->nw, &rho, u, &lam);
    real qq[2];
    cell_heatflux(c, h + (size_t)n * c->nv, b + (size_t)n * c->nv, u, qq);
    for (int i = 0; i < c->dim; i++) q[(size_t)n * c->dim + i] = qq[i];
  }
}

void or_maxwellian(const or_case* c, const real* W, real* h, real* b) {
#pragma omp parallel for schedule(static)
  for (int n = 0; n < c->ncell; n++) {
    real rho, u[2], lam;
    prim(c, W + (size_t)n * c->nw, &rho, u, &lam);
    for (int k = 0; k < c->nv; k++)
      maxw(c, rho, u, lam, c->vk_x[k], c->vk_y[k], &h[(size_t)n * c->nv + k], &b[(size_t)n * c->nv + k]);
  }
}

/* ------------------------------------------------------------------------ */
/* time steps (Sec. 2.2: dt_s with CFL 0.5, virtual step dt' with CFL 100)   */
/* ------------------------------------------------------------------------ */
/* per face: max_k |(v_k - U_f).n| */
static real face_smax(const or_case* c, const face_t* F) {
  real m = 0.0;
  for (int k = 0; k < c->nv; k++) {
    real wn = (c->vk_x[k] - F->ux) * F->nx + (c->vk_y[k] - F->uy) * F->ny;
    if (fabs(wn) > m) m = fabs(wn);
  }
  return m;
}
/* Reading: dt_s = CFL_s min over field cells of |Omega| / sum_f S_f smax_f / 2,
   dt'_i = CFL' |Omega_i| / sum_f S_f smax_f / 2. */
real or_timesteps(const or_case* c, real* dtp) {
  real* sm = (real*)malloc(sizeof(real) * (c->nface > 0 ? c->nface : 1));
  for (int f = 0; f < c->nface; f++) sm[f] = face_smax(c, &c->face[f]);
  real dts = INFINITY;
  for (int n = 0; n < c->ncell; n++) {
    real s = 0.0;
    for (int q = 0; q < 4; q++) {
      int f = c->cface[4 * n + q];
      if (f >= 0) s += 0.5 * c->face[f].S * sm[f];
    }
    if (dtp) dtp[n] = c->cfl_p * c->vol[n] / s;
    if (c->type[n] == OR_FIELD) {
      real t = c->cfl_s * c->vol[n] / s;
      if (t < dts) dts = t;
    }
  }
  free(sm);
  return dts;
}

/* ------------------------------------------------------------------------ */
/* reconstruction (Sec. 2.1: f0 = f^{l,r} + x . grad f^{l,r})                */
/* Reading: van Leer limiter per index direction, physical gradient through  */
/* the cell metric; one-sided difference beside a wall; zero when a          */
/* neighbour is a hole or missing; virtual ghost cells have zero slope.      */
/* ------------------------------------------------------------------------ */
static real vanleer(real s1, real s2) {
  if (s1 * s2 <= 0.0) return 0.0;
  return (s1 * fabs(s2) + fabs(s1) * s2) / (fabs(s1) + fabs(s2));
}

/* value accessor over f arrays (stride nv) or W arrays (stride nw) */
typedef struct { const real* a; const real* inf; int stride; } acc_t;
static real acc_get(const acc_t* A, nbref r, int cell, int m) {
  switch (r.kind) {
    case NB_CELL: return A->a[(size_t)r.cell * A->stride + m];
    case NB_FF: return A->inf[m];
    case NB_COPY: return A->a[(size_t)cell * A->stride + m];
    default: return 0.0;
  }
}
static real index_slope(const or_case* c, const acc_t* A, int cell, int dir, int m) {
  nbref lo = nbr(c, cell, dir, -1), hi = nbr(c, cell, dir, +1);
  if (lo.kind == NB_MISSING || hi.kind == NB_MISSING) return 0.0;
  real v0 = A->a[(size_t)cell * A->stride + m];
  if (lo.kind == NB_WALL && hi.kind == NB_WALL) return 0.0;
  if (lo.kind == NB_WALL) return acc_get(A, hi, cell, m) - v0;
  if (hi.kind == NB_WALL) return v0 - acc_get(A, lo, cell, m);
  return vanleer(v0 - acc_get(A, lo, cell, m), acc_get(A, hi, cell, m) - v0);
}
static void phys_grad(const or_case* c, const acc_t* A, int cell, int m, real* gx, real* gy) {
  real si = index_slope(c, A, cell, 0, m);
  real sj = (c->dim == 2) ? index_slope(c, A, cell, 1, m) : 0.0;
  const real* g = c->g + 4 * cell;
  *gx = g[0] * si + g[1] * sj;
  *gy = (c->dim == 2) ? g[2] * si + g[3] * sj : 0.0;
}

/* ------------------------------------------------------------------------ */
/* UGKS interface flux (Eqs. microscopicFlux, macroscopicFlux, fullSolution, */
/* maxWalldes; time average over dt_s)                                       */
/* ------------------------------------------------------------------------ */
typedef struct {
  int active;
  real rho, u[2], lam, q[2], tau;
  real a[2][4], A[4], tc[5];
  /* wall */
  real nwx, nwy, sgn;  /* normal into the wall, and +-1 face-normal sign */
  real rhow, lamw;
} frec_t;

typedef struct {
  const or_case* c;
  const real *h, *b, *W, *q;
  real* gW;     /* [ncell][2][nw] physical gradients of W */
  frec_t* rec;
  real dts;
} flux_ctx;

/* reconstructed value and gradient of f (h: comp 0, b: comp 1) from side s
   (0 = L, 1 = R) of face f at velocity k */
static void side_value(const flux_ctx* X, const face_t* F, int s, int k,
                       real* vh, real* vb, real* gh, real* gb) {
  const or_case* c = X->c;
  int cell = (s == 0) ? F->L : F->R;
  if (cell < 0) { /* virtual ghost, zero slope */
    if (F->gkind == NB_FF) { *vh = c->finf_h[k]; *vb = c->finf_b[k]; }
    else { *vh = X->h[(size_t)F->gcell * c->nv + k]; *vb = X->b[(size_t)F->gcell * c->nv + k]; }
    gh[0] = gh[1] = gb[0] = gb[1] = 0.0;
    return;
  }
  acc_t Ah = {X->h + k, c->finf_h + k, c->nv};
  acc_t Ab = {X->b + k, c->finf_b + k, c->nv};
  phys_grad(c, &Ah, cell, 0, &gh[0], &gh[1]);
  phys_grad(c, &Ab, cell, 0, &gb[0], &gb[1]);
  int slot = 2 * F->dir + ((s == 0) ? 1 : 0);
  real dx = c->cdx[8 * cell + 2 * slot], dy = c->cdx[8 * cell + 2 * slot + 1];
  *vh = X->h[(size_t)cell * c->nv + k] + gh[0] * dx + gh[1] * dy;
  *vb = X->b[(size_t)cell * c->nv + k] + gb[0] * dx + gb[1] * dy;
}

/* interface distribution integrated over [0, dts] (Eq. fullSolution) for the
   upwind data (fh, fb, gh, gb) and the equilibrium record R, at velocity k */
static void interface_integral(const or_case* c, const frec_t* R, const face_t* F, int k,
                               real fh, real fb, const real* gh, const real* gb,
                               real* Ih, real* Ib) {
  int d = c->dim;
  real vx = c->vk_x[k], vy = c->vk_y[k];
  real wx = vx - F->ux, wy = (d == 2) ? vy - F->uy : 0.0;
  real H, B, Hp, Bp;
  maxw(c, R->rho, R->u, R->lam, vx, vy, &H, &B);
  real v[2] = {vx, vy};
  or_shakhov(d, c->pr, R->rho, R->u, R->lam, R->q, v, &Hp, &Bp);
  real wah = wx * apsi(d, R->a[0], vx, vy, R->lam, 0);
  real wab = wx * apsi(d, R->a[0], vx, vy, R->lam, 1);
  if (d == 2) {
    wah += wy * apsi(d, R->a[1], vx, vy, R->lam, 0);
    wab += wy * apsi(d, R->a[1], vx, vy, R->lam, 1);
  }
  real Ah = apsi(d, R->A, vx, vy, R->lam, 0), Ab = apsi(d, R->A, vx, vy, R->lam, 1);
  real wgh = wx * gh[0] + wy * gh[1], wgb = wx * gb[0] + wy * gb[1];
  const real* t = R->tc;
  *Ih = t[0] * fh + t[1] * wgh + t[2] * (H + Hp) + t[3] * wah * H + t[4] * Ah * H;
  *Ib = t[0] * fb + t[1] * wgb + t[2] * (B + Bp) + t[3] * wab * B + t[4] * Ab * B;
}

static void set_coeffs(const or_case* c, frec_t* R, const real* uf, const real* dW, real dts) {
  real itau = inv_tau(c, R->rho, R->lam);
  R->tau = (itau == 0.0) ? INFINITY : 1.0 / itau;
  real a[8], A[4];
  or_slope_coeffs(c->dim, R->rho, R->u, R->lam, uf, dW, a, A);
  for (int d = 0; d < c->dim; d++)
    for (int m = 0; m < c->nw; m++) R->a[d][m] = a[d * c->nw + m];
  for (int m = 0; m < c->nw; m++) R->A[m] = A[m];
  or_time_coeffs(dts, R->tau, R->tc);
}

/* face equilibrium: W0 and q0 from the upwind interface data (reading: a tie
   wn = 0 takes the mean of both sides), slopes from the mean of the two cell
   gradients of W (ghost gradient zero). */
static void face_record(const flux_ctx* X, int f) {
  const or_case* c = X->c;
  const face_t* F = &c->face[f];
  frec_t* R = &X->rec[f];
  memset(R, 0, sizeof(*R));
  int d = c->dim, nw = c->nw;
  if (F->kind == F_WALL) {
    int cell = (F->L >= 0) ? F->L : F->R;
    if (c->type[cell] != OR_FIELD) return;
    R->active = 1;
    R->sgn = (F->R < 0) ? 1.0 : -1.0; /* wall on the R side: face normal points into the wall */
    R->nwx = R->sgn * F->nx; R->nwy = R->sgn * F->ny;
    /* incident state: one-sided extrapolation of W to the wall face */
    const real* gw = X->gW + (size_t)cell * 2 * nw;
    int slot = 2 * F->dir + ((F->L >= 0) ? 1 : 0);
    real Win[4], dx = c->cdx[8 * cell + 2 * slot], dy = c->cdx[8 * cell + 2 * slot + 1];
    for (int m = 0; m < nw; m++) Win[m] = X->W[(size_t)cell * nw + m] + gw[m] * dx + gw[nw + m] * dy;
    /* Reading (the paper is silent on positivity): an extrapolated state
       with non-positive density or internal energy is replaced by the cell
       state. */
    if (!physical(c, Win))
      for (int m = 0; m < nw; m++) Win[m] = X->W[(size_t)cell * nw + m];
    prim(c, Win, &R->rho, R->u, &R->lam);
    R->q[0] = X->q[(size_t)cell * d];
    R->q[1] = (d == 2) ? X->q[(size_t)cell * d + 1] : 0.0;
    real uf[2] = {F->ux, F->uy};
    set_coeffs(c, R, uf, gw, X->dts);
    /* wall density from zero net mass flux (Eq. maxWalldes) */
    R->lamw = 1.0 / (2.0 * F->rtw);
    real num = 0.0, den = 0.0;
    real nrm = pow(R->lamw / PI, 0.5 * d);
    for (int k = 0; k < c->nv; k++) {
      real vx = c->vk_x[k], vy = c->vk_y[k];
      real wn = (vx - F->ux) * R->nwx + (vy - F->uy) * R->nwy;
      if (wn > 0.0) {
        real fh, fb, gh[2], gb[2], Ih, Ib;
        side_value(X, F, (F->L >= 0) ? 0 : 1, k, &fh, &fb, gh, gb);
        interface_integral(c, R, F, k, fh, fb, gh, gb, &Ih, &Ib);
        num += c->wk[k] * wn * Ih;
      } else if (wn < 0.0) {
        real cx = vx - F->vwx, cy = (d == 2) ? vy - F->vwy : 0.0;
        den += c->wk[k] * wn * nrm * exp(-R->lamw * (cx * cx + cy * cy));
      }
    }
    R->rhow = -num / (X->dts * den);
    return;
  }
  int Lf = (F->L >= 0 && c->type[F->L] == OR_FIELD);
  int Rf = (F->R >= 0 && c->type[F->R] == OR_FIELD);
  if (!Lf && !Rf) return;
  R->active = 1;
  real W0[4] = {0, 0, 0, 0};
  for (int k = 0; k < c->nv; k++) {
    real vx = c->vk_x[k], vy = c->vk_y[k];
    real wn = (vx - F->ux) * F->nx + (vy - F->uy) * F->ny;
    real hl, bl, hr, br, g[2], gb[2], fh, fb;
    side_value(X, F, 0, k, &hl, &bl, g, gb);
    side_value(X, F, 1, k, &hr, &br, g, gb);
    if (wn > 0.0) { fh = hl; fb = bl; }
    else if (wn < 0.0) { fh = hr; fb = br; }
    else { fh = 0.5 * (hl + hr); fb = 0.5 * (bl + br); }
    real w = c->wk[k];
    W0[0] += w * fh;
    W0[1] += w * vx * fh;
    if (d == 2) W0[2] += w * vy * fh;
    W0[d + 1] += w * 0.5 * ((vx * vx + vy * vy) * fh + fb);
  }
  prim(c, W0, &R->rho, R->u, &R->lam);
  R->q[0] = R->q[1] = 0.0;
  for (int k = 0; k < c->nv; k++) {
    real vx = c->vk_x[k], vy = c->vk_y[k];
    real wn = (vx - F->ux) * F->nx + (vy - F->uy) * F->ny;
    real hl, bl, hr, br, g[2], gb[2], fh, fb;
    side_value(X, F, 0, k, &hl, &bl, g, gb);
    side_value(X, F, 1, k, &hr, &br, g, gb);
    if (wn > 0.0) { fh = hl; fb = bl; }
    else if (wn < 0.0) { fh = hr; fb = br; }
    else { fh = 0.5 * (hl + hr); fb = 0.5 * (bl + br); }
    real cx = vx - R->u[0], cy = (d == 2) ? vy - R->u[1] : 0.0;
    real e = (cx * cx + cy * cy) * fh + fb;
    R->q[0] += c->wk[k] * 0.5 * cx * e;
    if (d == 2) R->q[1] += c->wk[k] * 0.5 * cy * e;
  }
  real dW[8];
  for (int dd = 0; dd < 2; dd++)
    for (int m = 0; m < nw; m++) {
      real gl = (F->L >= 0) ? X->gW[(size_t)F->L * 2 * nw + dd * nw + m] : 0.0;
      real gr = (F->R >= 0) ? X->gW[(size_t)F->R * 2 * nw + dd * nw + m] : 0.0;
      dW[dd * nw + m] = 0.5 * (gl + gr);
    }
  real uf[2] = {F->ux, F->uy};
  set_coeffs(c, R, uf, dW, X->dts);
}

/* time-averaged flux along the face normal (L -> R) at velocity k */
static void face_flux_k(const flux_ctx* X, int f, int k, real* Fh, real* Fb) {
  const or_case* c = X->c;
  const face_t* F = &c->face[f];
  const frec_t* R = &X->rec[f];
  *Fh = *Fb = 0.0;
  if (!R->active) return;
  real vx = c->vk_x[k], vy = c->vk_y[k];
  if (F->kind == F_WALL) {
    real wn = (vx - F->ux) * R->nwx + (vy - F->uy) * R->nwy;
    real fh = 0.0, fb = 0.0;
    if (wn > 0.0) {
      real vh, vb, gh[2], gb[2], Ih, Ib;
      side_value(X, F, (F->L >= 0) ? 0 : 1, k, &vh, &vb, gh, gb);
      interface_integral(c, R, F, k, vh, vb, gh, gb, &Ih, &Ib);
      fh = wn * Ih / X->dts;
      fb = wn * Ib / X->dts;
    } else if (wn < 0.0) {
      real cx = vx - F->vwx, cy = (c->dim == 2) ? vy - F->vwy : 0.0;
      real Hw = R->rhow * pow(R->lamw / PI, 0.5 * c->dim) * exp(-R->lamw * (cx * cx + cy * cy));
      fh = wn * Hw;
      fb = wn * (real)c->nxi / (2.0 * R->lamw) * Hw;
    }
    *Fh = R->sgn * fh;
    *Fb = R->sgn * fb;
    return;
  }
  real wn = (vx - F->ux) * F->nx + (vy - F->uy) * F->ny;
  if (wn == 0.0) return;
  real vh, vb, gh[2], gb[2], Ih, Ib;
  side_value(X, F, (wn > 0.0) ? 0 : 1, k, &vh, &vb, gh, gb);
  interface_integral(c, R, F, k, vh, vb, gh, gb, &Ih, &Ib);
  *Fh = wn * Ih / X->dts;
  *Fb = wn * Ib / X->dts;
}

/* macro flux of face f (Eq. macroscopicFlux): velocity sums of Psi times
   the time-integrated interface flux */
static void face_macro(const flux_ctx* X, int f, real* Fm) {
  const or_case* c = X->c;
  for (int k = 0; k < c->nv; k++) {
    real fh, fb;
    face_flux_k(X, f, k, &fh, &fb);
    real vx = c->vk_x[k], vy = c->vk_y[k], w = c->wk[k];
    Fm[0] += w * fh;
    Fm[1] += w * vx * fh;
    if (c->dim == 2) Fm[2] += w * vy * fh;
    Fm[c->dim + 1] += w * 0.5 * ((vx * vx + vy * vy) * fh + fb);
  }
}

/* flux divergence of cell n, D = -(1/|Omega|) sum_f sigma S F, zero for a
   cell that is not a field cell */
static void cell_div(const flux_ctx* X, int n, real* dh, real* db) {
  const or_case* c = X->c;
  for (int k = 0; k < c->nv; k++) { dh[k] = 0.0; db[k] = 0.0; }
  if (c->type[n] != OR_FIELD) return;
  for (int s = 0; s < 4; s++) {
    int f = c->cface[4 * n + s];
    if (f < 0) continue;
    real sg = (real)c->csign[4 * n + s], S = c->face[f].S;
    for (int k = 0; k < c->nv; k++) {
      real fh, fb;
      face_flux_k(X, f, k, &fh, &fb);
      dh[k] -= sg * S * fh / c->vol[n];
      db[k] -= sg * S * fb / c->vol[n];
    }
  }
}

static void cell_grad_W(const or_case* c, const real* W, real* gW) {
#pragma omp parallel for schedule(static)
  for (int n = 0; n < c->ncell; n++) {
    real* g = gW + (size_t)n * 2 * c->nw;
    for (int m = 0; m < 2 * c->nw; m++) g[m] = 0.0;
    if (c->type[n] == OR_HOLE) continue;
    acc_t A = {W, c->winf, c->nw};
    for (int m = 0; m < c->nw; m++) phys_grad(c, &A, n, m, &g[m], &g[c->nw + m]);
  }
}

void or_flux(const or_case* c, real dts, const real* h, const real* b,
             const real* W, const real* q, real* Dh, real* Db,
             real* F, real* wall) {
  flux_ctx X = {c, h, b, W, q, NULL, NULL, dts};
  X.gW = (real*)malloc(sizeof(real) * 2 * c->nw * (size_t)c->ncell);
  X.rec = (frec_t*)calloc(c->nface > 0 ? c->nface : 1, sizeof(frec_t));
  cell_grad_W(c, W, X.gW);
#pragma omp parallel for schedule(dynamic, 4)
  for (int f = 0; f < c->nface; f++) face_record(&X, f);
  /* macro flux per face (Eq. macroscopicFlux) */
#pragma omp parallel for schedule(dynamic, 4)
  for (int f = 0; f < c->nface; f++) {
    real Fm[4] = {0, 0, 0, 0};
    face_macro(&X, f, Fm);
    for (int m = 0; m < c->nw; m++) F[(size_t)f * c->nw + m] = Fm[m];
    if (wall) {
      real* o = wall + (size_t)f * (1 + c->nw);
      for (int m = 0; m <= c->nw; m++) o[m] = 0.0;
      if (c->face[f].kind == F_WALL && X.rec[f].active) {
        o[0] = X.rec[f].rhow;
        for (int m = 0; m < c->nw; m++) o[1 + m] = X.rec[f].sgn * Fm[m];
      }
    }
  }
  /* divergence, gathered per cell: D = -(1/|Omega|) sum_f sigma S F */
#pragma omp parallel for schedule(dynamic, 4)
  for (int n = 0; n < c->ncell; n++)
    cell_div(&X, n, Dh + (size_t)n * c->nv, Db + (size_t)n * c->nv);
  free(X.gW);
  free(X.rec);
}

/* Wall loads (Sec. 2.1: the macro flux into an isothermal wall gives the
   load and the heat flux on the body).  Per wall face the flux into the wall
   per unit area: momentum (the load on the body), its component along the
   normal pointing into the wall (pressure) and along that normal turned by
   +90 degrees (shear), and energy; per block side the area integrals of the
   force, of its moment about the block's moved rotation centre and of the
   energy flux, summed in face order. */
void or_wall_loads(const or_case* c, const real* F, real* face_out, real* side_out) {
  int d = c->dim, nw = c->nw;
  if (face_out)
    for (size_t i = 0; i < (size_t)c->nface * (d + 3); i++) face_out[i] = 0.0;
  if (side_out)
    for (int i = 0; i < 16 * c->nblock; i++) side_out[i] = 0.0;
  for (int f = 0; f < c->nface; f++) {
    const face_t* Fc = &c->face[f];
    if (Fc->kind != F_WALL) continue;
    real sg = (Fc->R < 0) ? 1.0 : -1.0;  /* wall on the R side: the normal points into it */
    real nix = sg * Fc->nx, niy = sg * Fc->ny;
    real mx = sg * F[(size_t)f * nw + 1];
    real my = (d == 2) ? sg * F[(size_t)f * nw + 2] : 0.0;
    real en = sg * F[(size_t)f * nw + d + 1];
    if (face_out) {
      real* o = face_out + (size_t)f * (d + 3);
      o[0] = mx;
      if (d == 2) o[1] = my;
      o[d] = mx * nix + my * niy;
      o[d + 1] = -mx * niy + my * nix;
      o[d + 2] = en;
    }
    if (side_out) {
      const blk_t* B = &c->blk[Fc->blk];
      real rx = Fc->xf - (B->xc0 + B->dx), ry = Fc->yf - (B->yc0 + B->dy);
      real* o = side_out + 4 * (4 * Fc->blk + Fc->side);
      o[0] += Fc->S * mx;
      o[1] += Fc->S * my;
      o[2] += Fc->S * (rx * my - ry * mx);
      o[3] += Fc->S * en;
    }
  }
}

/* Newton-Euler (3-DOF) motion of block b (Sec. 3, Step 1: a body moves by
   the Newton-Euler equations or by a given motion).  Reading (loose
   coupling, the paper gives no integrator): the force and moment on the body
   at level n are the area integrals of the macro flux into the block's walls
   from the face macro flux F of the last flux evaluation (moment about the
   block's rotation centre, taken as the centre of mass), plus a constant
   external force and moment; the velocities take an explicit step and the
   pose the trapezoidal rule, exact for constant loads:
     u' = u + dt (F + F_ext) / m,   om' = om + dt (M + M_ext) / I,
     d' = d + dt (u + u') / 2,      th' = th + dt (om + om') / 2.
   body = {m, I, Fx_ext, Fy_ext, M_ext}; pose = {dx, dy, th, ux, uy, om} of
   the block, advanced in place (the caller sets the new pose). */
void or_newton_euler(const or_case* c, int b, const real* body, real dt, const real* F, real* pose) {
  real* side = (real*)malloc(sizeof(real) * 16 * c->nblock);
  or_wall_loads(c, F, NULL, side);
  real fx = body[2], fy = body[3], mz = body[4];
  for (int s = 0; s < 4; s++) {
    if (c->blk[b].bc[s] != OR_WALL) continue;
    fx += side[16 * b + 4 * s + 0];
    fy += side[16 * b + 4 * s + 1];
    mz += side[16 * b + 4 * s + 2];
  }
  free(side);
  real ux = pose[3] + dt * fx / body[0];
  real uy = pose[4] + dt * fy / body[0];
  real om = pose[5] + dt * mz / body[1];
  pose[0] += 0.5 * dt * (pose[3] + ux);
  pose[1] += 0.5 * dt * (pose[4] + uy);
  pose[2] += 0.5 * dt * (pose[5] + om);
  pose[3] = ux; pose[4] = uy; pose[5] = om;
}

/* ------------------------------------------------------------------------ */
/* overset interpolation (Sec. 3.2) -- weights supplied by the assembly      */
/* ------------------------------------------------------------------------ */
/* rows r0 .. r0+nrow-1 of the donor table; their donors are not rows of
   the same call, so the rows are independent */
static void interp_rows(const or_case* c, int r0, int nrow, real* h, real* b, real* W, real* q) {
#pragma omp parallel for schedule(static)
  for (int r = r0; r < r0 + nrow; r++) {
    int n = c->rec[r];
    for (int k = 0; k < c->nv; k++) {
      real sh = 0.0, sb = 0.0;
      for (int p = c->dptr[r]; p < c->dptr[r + 1]; p++) {
        sh += c->dw[p] * h[(size_t)c->don[p] * c->nv + k];
        sb += c->dw[p] * b[(size_t)c->don[p] * c->nv + k];
      }
      h[(size_t)n * c->nv + k] = sh;
      b[(size_t)n * c->nv + k] = sb;
    }
    for (int m = 0; m < c->nw; m++) {
      real s = 0.0;
      for (int p = c->dptr[r]; p < c->dptr[r + 1]; p++) s += c->dw[p] * W[(size_t)c->don[p] * c->nw + m];
      W[(size_t)n * c->nw + m] = s;
    }
    if (q)
      for (int m = 0; m < c->dim; m++) {
        real s = 0.0;
        for (int p = c->dptr[r]; p < c->dptr[r + 1]; p++) s += c->dw[p] * q[(size_t)c->don[p] * c->dim + m];
        q[(size_t)n * c->dim + m] = s;
      }
  }
}

void or_interp(const or_case* c, real* h, real* b, real* W, real* q) {
  interp_rows(c, 0, c->nrec, h, b, W, q);
}

/* ------------------------------------------------------------------------ */
/* dual time stepping (Sec. 2.2)                                             */
/* ------------------------------------------------------------------------ */
/* Shakhov equilibrium h+ = H + H+, b+ = B + B+ of (W, q) at velocity k */
static void fplus(const or_case* c, real rho, const real* u, real lam, const real* q,
                  int k, real* hp, real* bp) {
  real H, B, Hs, Bs, v[2] = {c->vk_x[k], c->vk_y[k]};
  maxw(c, rho, u, lam, v[0], v[1], &H, &B);
  or_shakhov(c->dim, c->pr, rho, u, lam, q, v, &Hs, &Bs);
  *hp = H + Hs;
  *bp = B + Bs;
}

/* S = f^n/dt + r^n/2 of cell n, r^n = D^n + (f+^n - f^n)/tau^n
   (Eq. residual_macro_n); h, b, dh, db, sh, sb are the cell's rows; zero
   outside the field cells */
static void cell_source(const or_case* c, real dt, int n, const real* h, const real* b,
                        const real* W, const real* q, const real* dh, const real* db,
                        real* sh, real* sb) {
  if (c->type[n] != OR_FIELD) {
    for (int k = 0; k < c->nv; k++) { sh[k] = 0.0; sb[k] = 0.0; }
    return;
  }
  real rho, u[2], lam, qq[2] = {0, 0};
  prim(c, W + (size_t)n * c->nw, &rho, u, &lam);
  for (int i = 0; i < c->dim; i++) qq[i] = q[(size_t)n * c->dim + i];
  real it = inv_tau(c, rho, lam);
  for (int k = 0; k < c->nv; k++) {
    real hp, bp;
    fplus(c, rho, u, lam, qq, k, &hp, &bp);
    sh[k] = h[k] / dt + 0.5 * (dh[k] + (hp - h[k]) * it);
    sb[k] = b[k] / dt + 0.5 * (db[k] + (bp - b[k]) * it);
  }
}

/* Steps 1-2: S = f^n/dt + r^n/2 at every cell, and the level-n face flux */
void or_begin_step(or_case* c, real dt, real dts, real* h, real* b,
                   real* W, real* q, real* Sh, real* Sb, real* Fn) {
  size_t N = (size_t)c->ncell * c->nv;
  real* Dh = (real*)malloc(sizeof(real) * N);
  real* Db = (real*)malloc(sizeof(real) * N);
  /* once after an assembly the cells uncovered from holes (their donors
     are cells that were live), then the receptors (which may use them) */
  interp_rows(c, c->nrec, c->nref, h, b, W, q);
  c->nref = 0;
  interp_rows(c, 0, c->nrec, h, b, W, q);
  or_flux(c, dts, h, b, W, q, Dh, Db, Fn, NULL);
#pragma omp parallel for schedule(static)
  for (int n = 0; n < c->ncell; n++) {
    size_t o = (size_t)n * c->nv;
    cell_source(c, dt, n, h + o, b + o, W, q, Dh + o, Db + o, Sh + o, Sb + o);
  }
  free(Dh); free(Db);
}

/* Steps 1-2 at a sample of cells only: the same interpolation into the
   rows of the donor table (over the whole field), then for each listed cell
   its flux divergence and S (rows [ns][nv]) and the macro flux of each of its
   four face slots (Fc [ns][4][nw], zero where a slot has no face).  The
   face records are formed only for the faces of the listed cells, so a
   sample of a large case costs little beyond the interpolation. */
void or_begin_step_cells(or_case* c, real dt, real dts, real* h, real* b, real* W, real* q,
                         int ns, const int* cells, real* Sh, real* Sb, real* Fc) {
  interp_rows(c, c->nrec, c->nref, h, b, W, q);
  c->nref = 0;
  interp_rows(c, 0, c->nrec, h, b, W, q);
  flux_ctx X = {c, h, b, W, q, NULL, NULL, dts};
  X.gW = (real*)malloc(sizeof(real) * 2 * c->nw * (size_t)c->ncell);
  X.rec = (frec_t*)calloc(c->nface > 0 ? c->nface : 1, sizeof(frec_t));
  cell_grad_W(c, W, X.gW);
  for (int i = 0; i < ns; i++)
    for (int s = 0; s < 4; s++) {
      int f = c->cface[4 * cells[i] + s];
      if (f >= 0) face_record(&X, f);
    }
#pragma omp parallel for schedule(dynamic, 1)
  for (int i = 0; i < ns; i++) {
    int n = cells[i];
    real* dh = (real*)malloc(sizeof(real) * 2 * (size_t)c->nv);
    real* db = dh + c->nv;
    cell_div(&X, n, dh, db);
    cell_source(c, dt, n, h + (size_t)n * c->nv, b + (size_t)n * c->nv, W, q, dh, db,
                Sh + (size_t)i * c->nv, Sb + (size_t)i * c->nv);
    for (int s = 0; s < 4; s++) {
      real Fm[4] = {0, 0, 0, 0};
      int f = c->cface[4 * n + s];
      if (f >= 0) face_macro(&X, f, Fm);
      for (int m = 0; m < c->nw; m++) Fc[((size_t)i * 4 + s) * c->nw + m] = Fm[m];
    }
    free(dh);
  }
  free(X.gW);
  free(X.rec);
}

/* ALE Euler flux F_E(W; n, U) = (rho th, rho V th + p n, rho E th + p V.n),
   th = (V - U).n */
static void euler_flux(const or_case* c, const real* W, real nx, real ny,
                       real ux, real uy, real* Fe) {
  real rho, u[2], lam;
  prim(c, W, &rho, u, &lam);
  real p = rho / (2.0 * lam);
  int d = c->dim;
  real th = (u[0] - ux) * nx + ((d == 2) ? (u[1] - uy) * ny : 0.0);
  Fe[0] = rho * th;
  Fe[1] = W[1] * th + p * nx;
  if (d == 2) Fe[2] = W[2] * th + p * ny;
  Fe[d + 1] = W[d + 1] * th + p * (u[0] * nx + ((d == 2) ? u[1] * ny : 0.0));
}

static real sound(const or_case* c, const real* W) {
  real rho, u[2], lam;
  prim(c, W, &rho, u, &lam);
  real gam = (real)(c->dim + c->nxi + 2) / (real)(c->dim + c->nxi);
  return sqrt(gam / (2.0 * lam));
}

/* W of the neighbour across face slot s of cell n, for the spectral radius */
static const real* nb_W(const or_case* c, const real* W, int n, int s) {
  int f = c->cface[4 * n + s];
  const face_t* F = &c->face[f];
  if (F->kind == F_GHOST) return (F->gkind == NB_FF) ? c->winf : W + (size_t)F->gcell * c->nw;
  int o = (F->L == n) ? F->R : F->L;
  return W + (size_t)o * c->nw;
}

/* spectral radius Gamma of the face in slot s of cell n (Sec. 2.2; reading:
   arithmetic means of both sides; a wall face uses the cell alone) */
static real face_gamma(const or_case* c, const real* W, int n, int s) {
  int f = c->cface[4 * n + s];
  const face_t* F = &c->face[f];
  const real* Wi = W + (size_t)n * c->nw;
  real ri, ui[2], li;
  prim(c, Wi, &ri, ui, &li);
  real ai = sound(c, Wi);
  if (F->kind == F_WALL) {
    real th = (ui[0] - F->ux) * F->nx + ((c->dim == 2) ? (ui[1] - F->uy) * F->ny : 0.0);
    return fabs(th) + ai;
  }
  const real* Wj = nb_W(c, W, n, s);
  real rj, uj[2], lj;
  prim(c, Wj, &rj, uj, &lj);
  real aj = sound(c, Wj);
  real mx = 0.5 * (ui[0] + uj[0]), my = 0.5 * (ui[1] + uj[1]);
  real th = (mx - F->ux) * F->nx + ((c->dim == 2) ? (my - F->uy) * F->ny : 0.0);
  return fabs(th) + 0.5 * (ai + aj);
}

/* the field neighbour in slot s of cell n in the same block, or -1 */
static int field_nb(const or_case* c, int n, int s) {
  int f = c->cface[4 * n + s];
  if (f < 0) return -1;
  const face_t* F = &c->face[f];
  if (F->kind != F_INTERIOR) return -1;
  int o = (F->L == n) ? F->R : F->L;
  return (c->type[o] == OR_FIELD) ? o : -1;
}

/*
 * Step 4: macro delta form (Eq. dualTimeStepping_macro) solved by LU-SGS with
 * the Euler-flux approximation of dF and the spectral radius Gamma.  The
 * cell's own dF_E term cancels (sum_f S n = 0 and sum_f S U.n = 0 for a rigid
 * cell).  Order: ascending global cell index (lexicographic per block).
 */
void or_macro_lusgs(const or_case* c, real dt, const real* dtp, const real* W,
                    const real* Wn, const real* F, const real* Fn, real* Wp,
                    real* resid) {
  int nw = c->nw;
  size_t NW = (size_t)c->ncell * nw;
  real* R = (real*)calloc(NW, sizeof(real));
  real* Dg = (real*)calloc(c->ncell, sizeof(real));
  real* dWs = (real*)calloc(NW, sizeof(real));
  real* dW = (real*)calloc(NW, sizeof(real));
  real rs[4] = {0, 0, 0, 0};
  for (int n = 0; n < c->ncell; n++) {
    if (c->type[n] != OR_FIELD) continue;
    real sg = 0.0;
    for (int m = 0; m < nw; m++) R[n * nw + m] = -(W[n * nw + m] - Wn[n * nw + m]) / dt;
    for (int s = 0; s < 4; s++) {
      int f = c->cface[4 * n + s];
      if (f < 0) continue;
      real S = c->face[f].S, sig = (real)c->csign[4 * n + s];
      for (int m = 0; m < nw; m++)
        R[n * nw + m] -= sig * S * (F[(size_t)f * nw + m] + Fn[(size_t)f * nw + m]) / (2.0 * c->vol[n]);
      sg += S * face_gamma(c, W, n, s);
    }
    Dg[n] = 1.0 / dtp[n] + 1.0 / dt + sg / (4.0 * c->vol[n]);
    for (int m = 0; m < nw; m++) rs[m] += R[n * nw + m] * R[n * nw + m];
  }
  if (resid) for (int m = 0; m < nw; m++) resid[m] = sqrt(rs[m]);
  /* forward sweep */
  for (int n = 0; n < c->ncell; n++) {
    if (c->type[n] != OR_FIELD) continue;
    real acc[4] = {0, 0, 0, 0};
    for (int s = 0; s < 4; s++) {
      int j = field_nb(c, n, s);
      if (j < 0 || j >= n) continue;
      int f = c->cface[4 * n + s];
      const face_t* Fc = &c->face[f];
      real sig = (real)c->csign[4 * n + s];
      real nx = sig * Fc->nx, ny = sig * Fc->ny;
      real Wt[4], F1[4], F0[4];
      for (int m = 0; m < nw; m++) Wt[m] = W[j * nw + m] + dWs[j * nw + m];
      euler_flux(c, Wt, nx, ny, Fc->ux, Fc->uy, F1);
      euler_flux(c, W + (size_t)j * nw, nx, ny, Fc->ux, Fc->uy, F0);
      real G = face_gamma(c, W, n, s);
      for (int m = 0; m < nw; m++) acc[m] += Fc->S * ((F1[m] - F0[m]) - G * dWs[j * nw + m]);
    }
    for (int m = 0; m < nw; m++)
      dWs[n * nw + m] = (R[n * nw + m] - acc[m] / (4.0 * c->vol[n])) / Dg[n];
  }
  /* backward sweep */
  for (int n = c->ncell - 1; n >= 0; n--) {
    if (c->type[n] != OR_FIELD) continue;
    real acc[4] = {0, 0, 0, 0};
    for (int s = 0; s < 4; s++) {
      int j = field_nb(c, n, s);
      if (j < 0 || j <= n) continue;
      int f = c->cface[4 * n + s];
      const face_t* Fc = &c->face[f];
      real sig = (real)c->csign[4 * n + s];
      real nx = sig * Fc->nx, ny = sig * Fc->ny;
      real Wt[4], F1[4], F0[4];
      for (int m = 0; m < nw; m++) Wt[m] = W[j * nw + m] + dW[j * nw + m];
      euler_flux(c, Wt, nx, ny, Fc->ux, Fc->uy, F1);
      euler_flux(c, W + (size_t)j * nw, nx, ny, Fc->ux, Fc->uy, F0);
      real G = face_gamma(c, W, n, s);
      for (int m = 0; m < nw; m++) acc[m] += Fc->S * ((F1[m] - F0[m]) - G * dW[j * nw + m]);
    }
    for (int m = 0; m < nw; m++)
      dW[n * nw + m] = dWs[n * nw + m] - acc[m] / (4.0 * c->vol[n] * Dg[n]);
  }
  for (size_t i = 0; i < NW; i++) Wp[i] = W[i] + dW[i];
  /* Reading (the paper is silent on positivity): a predictor with
     non-positive density or internal energy keeps the current state. */
  for (int n = 0; n < c->ncell; n++)
    if (c->type[n] == OR_FIELD && !physical(c, Wp + (size_t)n * nw))
      for (int m = 0; m < nw; m++) Wp[(size_t)n * nw + m] = W[(size_t)n * nw + m];
  free(R); free(Dg); free(dWs); free(dW);
}

/*
 * Steps 5-6: micro delta form (Eq. dualTimeStepping_micro), independent per
 * velocity, solved by LU-SGS with the upwind approximation of the flux
 * variation.  r = S - f^s/dt + (D^s + (f+' - f^s)/tau')/2, with tau' and f+'
 * from W' and q' (q' = heat flux of f^s about the velocity of W').
 * Neighbours that are not field cells of the same block are explicit.
 * On return h, b hold f^{s+1}.
 */
void or_micro_lusgs(const or_case* c, real dt, const real* dtp, const real* Wp,
                    const real* qp, real* h, real* b, const real* Sh,
                    const real* Sb, const real* Dh, const real* Db) {
  int nv = c->nv;
  real* crho = (real*)malloc(sizeof(real) * c->ncell);
  real* cu = (real*)malloc(sizeof(real) * 2 * c->ncell);
  real* clam = (real*)malloc(sizeof(real) * c->ncell);
  real* citau = (real*)malloc(sizeof(real) * c->ncell);
  for (int n = 0; n < c->ncell; n++) {
    prim(c, Wp + (size_t)n * c->nw, &crho[n], cu + 2 * n, &clam[n]);
    citau[n] = inv_tau(c, crho[n], clam[n]);
  }
#pragma omp parallel
  {
    real* xs_h = (real*)malloc(sizeof(real) * c->ncell);
    real* xs_b = (real*)malloc(sizeof(real) * c->ncell);
    real* dd = (real*)malloc(sizeof(real) * c->ncell);
#pragma omp for schedule(static)
    for (int k = 0; k < nv; k++) {
      real vx = c->vk_x[k], vy = c->vk_y[k];
      /* forward sweep: (D + L) df* = r */
      for (int n = 0; n < c->ncell; n++) {
        xs_h[n] = 0.0; xs_b[n] = 0.0;
        if (c->type[n] != OR_FIELD) continue;
        size_t o = (size_t)n * nv + k;
        real qq[2] = {qp[(size_t)n * c->dim], (c->dim == 2) ? qp[(size_t)n * c->dim + 1] : 0.0};
        real hp, bp;
        fplus(c, crho[n], cu + 2 * n, clam[n], qq, k, &hp, &bp);
        real rh = Sh[o] - h[o] / dt + 0.5 * (Dh[o] + (hp - h[o]) * citau[n]);
        real rb = Sb[o] - b[o] / dt + 0.5 * (Db[o] + (bp - b[o]) * citau[n]);
        real diag = 1.0 / dtp[n] + 1.0 / dt + 0.5 * citau[n];
        real offh = 0.0, offb = 0.0;
        for (int s = 0; s < 4; s++) {
          int f = c->cface[4 * n + s];
          if (f < 0) continue;
          const face_t* F = &c->face[f];
          real sig = (real)c->csign[4 * n + s];
          real wn = sig * ((vx - F->ux) * F->nx + (vy - F->uy) * F->ny);
          diag += F->S * ((wn > 0.0) ? wn : 0.0) / (2.0 * c->vol[n]);
          int j = field_nb(c, n, s);
          if (j < 0 || j >= n) continue;
          real wm = (wn < 0.0) ? wn : 0.0;
          offh += F->S * wm * xs_h[j];
          offb += F->S * wm * xs_b[j];
        }
        dd[n] = diag;
        xs_h[n] = (rh - offh / (2.0 * c->vol[n])) / diag;
        xs_b[n] = (rb - offb / (2.0 * c->vol[n])) / diag;
      }
      /* backward sweep: (D + U) df = D df* ; overwrite xs with df */
      for (int n = c->ncell - 1; n >= 0; n--) {
        if (c->type[n] != OR_FIELD) continue;
        real offh = 0.0, offb = 0.0;
        for (int s = 0; s < 4; s++) {
          int j = field_nb(c, n, s);
          if (j < 0 || j <= n) continue;
          int f = c->cface[4 * n + s];
          const face_t* F = &c->face[f];
          real sig = (real)c->csign[4 * n + s];
          real wn = sig * ((vx - F->ux) * F->nx + (vy - F->uy) * F->ny);
          real wm = (wn < 0.0) ? wn : 0.0;
          offh += F->S * wm * xs_h[j];
          offb += F->S * wm * xs_b[j];
        }
        xs_h[n] = xs_h[n] - offh / (2.0 * c->vol[n] * dd[n]);
        xs_b[n] = xs_b[n] - offb / (2.0 * c->vol[n] * dd[n]);
      }
      for (int n = 0; n < c->ncell; n++) {
        if (c->type[n] != OR_FIELD) continue;
        h[(size_t)n * nv + k] += xs_h[n];
        b[(size_t)n * nv + k] += xs_b[n];
      }
    }
    free(xs_h); free(xs_b); free(dd);
  }
  free(crho); free(cu); free(clam); free(citau);
}

/* Step 7 (reading of the garbled formula): W^{s+1} = W' + sum_k V_k Psi_k
   (f^{s+1} - g(W')), g the plain Maxwellian of W' */
void or_step7(const or_case* c, const real* Wp, const real* h, const real* b, real* W) {
#pragma omp parallel for schedule(static)
  for (int n = 0; n < c->ncell; n++) {
    const real* wp = Wp + (size_t)n * c->nw;
    real* w = W + (size_t)n * c->nw;
    if (c->type[n] != OR_FIELD) { for (int m = 0; m < c->nw; m++) w[m] = wp[m]; continue; }
    real rho, u[2], lam;
    prim(c, wp, &rho, u, &lam);
    real s[4] = {0, 0, 0, 0};
    int d = c->dim;
    for (int k = 0; k < c->nv; k++) {
      real H, B;
      real vx = c->vk_x[k], vy = c->vk_y[k];
      maxw(c, rho, u, lam, vx, vy, &H, &B);
      real dh = h[(size_t)n * c->nv + k] - H, db = b[(size_t)n * c->nv + k] - B;
      real wk = c->wk[k];
      s[0] += wk * dh;
      s[1] += wk * vx * dh;
      if (d == 2) s[2] += wk * vy * dh;
      s[d + 1] += wk * 0.5 * ((vx * vx + vy * vy) * dh + db);
    }
    for (int m = 0; m < c->nw; m++) w[m] = wp[m] + s[m];
  }
}

/* Steps 3-7: one inner iteration of the dual time stepping */
void or_pseudo_step(const or_case* c, real dt, real dts, const real* dtp,
                    real* h, real* b, real* W, const real* Wn, real* q,
                    const real* Sh, const real* Sb, const real* Fn,
                    real* resid, real* Fout) {
  size_t N = (size_t)c->ncell * c->nv, NW = (size_t)c->ncell * c->nw;
  real* Dh = (real*)malloc(sizeof(real) * N);
  real* Db = (real*)malloc(sizeof(real) * N);
  real* F = (real*)malloc(sizeof(real) * (size_t)(c->nface > 0 ? c->nface : 1) * c->nw);
  real* Wp = (real*)malloc(sizeof(real) * NW);
  real* qp = (real*)malloc(sizeof(real) * (size_t)c->ncell * c->dim);
  or_interp(c, h, b, W, q);                                  /* receptors first */
  or_flux(c, dts, h, b, W, q, Dh, Db, F, NULL);              /* Step 3 */
  if (Fout) memcpy(Fout, F, sizeof(real) * (size_t)c->nface * c->nw);
  or_macro_lusgs(c, dt, dtp, W, Wn, F, Fn, Wp, resid);       /* Step 4 */
  or_heatflux(c, h, b, Wp, qp);                              /* q' from f^s about V' */
  or_micro_lusgs(c, dt, dtp, Wp, qp, h, b, Sh, Sb, Dh, Db);  /* Steps 5-6 */
  or_step7(c, Wp, h, b, W);                                  /* Step 7 */
  or_heatflux(c, h, b, W, q);                                /* q^{s+1} */
  free(Dh); free(Db); free(F); free(Wp); free(qp);
}

/* ------------------------------------------------------------------------ */
/* overset assembly (Sec. 3.1) and interpolation weights (Sec. 3.2).        */
/* Brute force: every node is tested against every cell of the other zones  */
/* and every wall segment.  Each block is one grid zone.  Geometric          */
/* predicates use the fixed expressions below (no contraction), so that the  */
/* integer results are reproducible bit for bit:                             */
/*   point in quad:  all edge cross products (q_{k+1} - q_k) x (p - q_k) of  */
/*                   one sign or zero (edges and corners count as inside);   */
/*   wall distance:  squared distance to the nearest wall segment of the     */
/*                   zone, +inf for a zone without walls;                    */
/*   inside a body:  crossing number against each closed wall polygon of     */
/*                   the other zones (half-open in y).                       */
/* ------------------------------------------------------------------------ */
static int quad_contains(const real* qx, const real* qy, real px, real py) {
  int pos = 0, neg = 0;
  for (int k = 0; k < 4; k++) {
    int k1 = (k + 1) % 4;
    real cr = (qx[k1] - qx[k]) * (py - qy[k]) - (qy[k1] - qy[k]) * (px - qx[k]);
    if (cr > 0.0) pos = 1;
    if (cr < 0.0) neg = 1;
  }
  return !(pos && neg);
}

static void cell_quad(const or_case* c, int n, real* qx, real* qy) {
  int b = c->cblk[n], i = c->ci[n], j = c->cj[n];
  qx[0] = node_x(c, b, i, j);         qy[0] = node_y(c, b, i, j);
  qx[1] = node_x(c, b, i + 1, j);     qy[1] = node_y(c, b, i + 1, j);
  qx[2] = node_x(c, b, i + 1, j + 1); qy[2] = node_y(c, b, i + 1, j + 1);
  qx[3] = node_x(c, b, i, j + 1);     qy[3] = node_y(c, b, i, j + 1);
}

static real seg_dist2(real px, real py, real ax, real ay, real bx, real by) {
  real ex = bx - ax, ey = by - ay;
  real l2 = ex * ex + ey * ey;
  real t = 0.0;
  if (l2 > 0.0) {
    t = ((px - ax) * ex + (py - ay) * ey) / l2;
    if (t < 0.0) t = 0.0;
    if (t > 1.0) t = 1.0;
  }
  real dx = px - (ax + t * ex), dy = py - (ay + t * ey);
  return dx * dx + dy * dy;
}

/* the nodes of wall side s of block b, in order along the side */
static int side_nodes(const or_case* c, int b, int s, real* x, real* y) {
  const blk_t* B = &c->blk[b];
  int n = (s < 2) ? B->nj + 1 : B->ni + 1;
  for (int m = 0; m < n; m++) {
    int i = (s == 0) ? 0 : (s == 1) ? B->ni : m;
    int j = (s == 2) ? 0 : (s == 3) ? B->nj : m;
    x[m] = node_x(c, b, i, j);
    y[m] = node_y(c, b, i, j);
  }
  return n;
}

/* a wall side closes into a body outline when the block is periodic along it */
static int side_closed(const or_case* c, int b, int s) {
  const blk_t* B = &c->blk[b];
  return (s < 2) ? B->bc[2] == OR_PERIODIC : B->bc[0] == OR_PERIODIC;
}

static real wall_dist2(const or_case* c, int b, real px, real py, real* bx, real* by) {
  real d2 = INFINITY;
  for (int s = 0; s < 4; s++) {
    if (c->blk[b].bc[s] != OR_WALL) continue;
    int n = side_nodes(c, b, s, bx, by);
    for (int m = 0; m + 1 < n; m++) {
      real e = seg_dist2(px, py, bx[m], by[m], bx[m + 1], by[m + 1]);
      if (e < d2) d2 = e;
    }
  }
  return d2;
}

static int inside_body(const or_case* c, int self, real px, real py, real* bx, real* by) {
  for (int b = 0; b < c->nblock; b++) {
    if (b == self) continue;
    for (int s = 0; s < 4; s++) {
      if (c->blk[b].bc[s] != OR_WALL || !side_closed(c, b, s)) continue;
      int n = side_nodes(c, b, s, bx, by);
      int in = 0;
      for (int m = 0; m + 1 < n; m++) {
        real ax = bx[m], ay = by[m], ex = bx[m + 1], ey = by[m + 1];
        if ((ay > py) != (ey > py)) {
          real xi = ax + (py - ay) * (ex - ax) / (ey - ay);
          if (px < xi) in = !in;
        }
      }
      if (in) return 1;
    }
  }
  return 0;
}

/* cell layers between cell n and the nearest overset (no-face) side of its
   block; a large number for a block without such a side */
static int overset_depth(const or_case* c, int n) {
  const blk_t* B = &c->blk[c->cblk[n]];
  int i = c->ci[n], j = c->cj[n], d = 1 << 30;
  if (B->bc[0] == OR_NONE && i < d) d = i;
  if (B->bc[1] == OR_NONE && B->ni - 1 - i < d) d = B->ni - 1 - i;
  if (B->bc[2] == OR_NONE && j < d) d = j;
  if (B->bc[3] == OR_NONE && B->nj - 1 - j < d) d = B->nj - 1 - j;
  return d;
}

/* lowest cell of block b containing (px, py), restricted to field cells
   when `types` is given; -1 if none */
static int containing_cell(const or_case* c, int b, real px, real py, const int8_t* types) {
  const blk_t* B = &c->blk[b];
  real qx[4], qy[4];
  for (int n = B->cell0; n < B->cell0 + B->ni * B->nj; n++) {
    if (types && types[n] != OR_FIELD) continue;
    cell_quad(c, n, qx, qy);
    if (quad_contains(qx, qy, px, py)) return n;
  }
  return -1;
}

/* index neighbour of cell n along dir (0: i, 1: j), side -1 / +1, inside
   its block (periodic wrap), or -1 */
static int index_nb(const or_case* c, int n, int dir, int side) {
  int b = c->cblk[n], i = c->ci[n], j = c->cj[n];
  const blk_t* B = &c->blk[b];
  if (dir == 0) {
    i += side;
    if (i < 0 || i >= B->ni) {
      if (B->bc[0] != OR_PERIODIC) return -1;
      i = (i + B->ni) % B->ni;
    }
  } else {
    j += side;
    if (j < 0 || j >= B->nj) {
      if (B->bc[2] != OR_PERIODIC) return -1;
      j = (j + B->nj) % B->nj;
    }
  }
  return cell_index(c, b, i, j);
}

/* bilinear weights of (px, py) in the quad of cell centres n[0..3] (Newton
   for the inverse bilinear map, three steps from the middle) */
static void bilinear(const or_case* c, const int* n, real px, real py, real* w) {
  real x0 = c->cx[n[0]], x1 = c->cx[n[1]], x2 = c->cx[n[2]], x3 = c->cx[n[3]];
  real y0 = c->cy[n[0]], y1 = c->cy[n[1]], y2 = c->cy[n[2]], y3 = c->cy[n[3]];
  real s = 0.5, t = 0.5;
  for (int it = 0; it < 3; it++) {
    real rx = (1.0 - s) * (1.0 - t) * x0 + s * (1.0 - t) * x1 + s * t * x2 + (1.0 - s) * t * x3 - px;
    real ry = (1.0 - s) * (1.0 - t) * y0 + s * (1.0 - t) * y1 + s * t * y2 + (1.0 - s) * t * y3 - py;
    real xs = (1.0 - t) * (x1 - x0) + t * (x2 - x3), ys = (1.0 - t) * (y1 - y0) + t * (y2 - y3);
    real xt = (1.0 - s) * (x3 - x0) + s * (x2 - x1), yt = (1.0 - s) * (y3 - y0) + s * (y2 - y1);
    real det = xs * yt - xt * ys;
    s -= (rx * yt - xt * ry) / det;
    t -= (xs * ry - rx * ys) / det;
  }
  w[0] = (1.0 - s) * (1.0 - t); w[1] = s * (1.0 - t); w[2] = s * t; w[3] = (1.0 - s) * t;
}

/* donors and weights of cell n (Sec. 3.2): the field cell of another zone
   containing its centroid (lowest zone, then lowest cell); bilinear over the
   quad of donor-grid centroids around it (wrule 1, when such a quad of field
   cells contains it), else inverse distance squared over the donor and its
   field index neighbours.  Returns the donor count, or -1 if none. */
static int donors_of(const or_case* c, const int8_t* ty, int n, int wrule, int* don, real* w) {
  real px = c->cx[n], py = c->cy[n];
  int d = -1;
  for (int z = 0; z < c->nblock && d < 0; z++)
    if (z != c->cblk[n]) d = containing_cell(c, z, px, py, ty);
  if (d < 0) return -1;
  if (wrule == 1) {
    /* dual quads with the donor as a corner, in a fixed order */
    for (int q = 0; q < 4; q++) {
      int a = q % 2, bb = q / 2;
      int lo_i = (a == 0) ? index_nb(c, d, 0, -1) : d;
      int c00 = (lo_i < 0) ? -1 : ((bb == 0) ? index_nb(c, lo_i, 1, -1) : lo_i);
      if (c00 < 0) continue;
      int c10 = index_nb(c, c00, 0, +1);
      int c01 = index_nb(c, c00, 1, +1);
      int c11 = (c10 < 0) ? -1 : index_nb(c, c10, 1, +1);
      int nq[4] = {c00, c10, c11, c01};
      int ok = 1;
      for (int k = 0; k < 4; k++) ok = ok && nq[k] >= 0 && ty[nq[k]] == OR_FIELD;
      if (!ok) continue;
      real qx[4], qy[4];
      for (int k = 0; k < 4; k++) { qx[k] = c->cx[nq[k]]; qy[k] = c->cy[nq[k]]; }
      if (!quad_contains(qx, qy, px, py)) continue;
      bilinear(c, nq, px, py, w);
      for (int k = 0; k < 4; k++) don[k] = nq[k];
      return 4;
    }
  }
  int set[5], ns = 0;
  set[ns++] = d;
  for (int dir = 0; dir < 2; dir++)
    for (int sd = -1; sd <= 1; sd += 2) {
      int m = index_nb(c, d, dir, sd), dup = 0;
      if (m < 0 || ty[m] != OR_FIELD) continue;
      for (int k = 0; k < ns; k++) dup = dup || set[k] == m;
      if (!dup) set[ns++] = m;
    }
  real d2[5];
  int exact = -1;
  for (int k = 0; k < ns; k++) {
    real dx = c->cx[set[k]] - px, dy = c->cy[set[k]] - py;
    d2[k] = dx * dx + dy * dy;
    if (exact < 0 && d2[k] <= 1e-28 * c->vol[set[k]]) exact = k;
  }
  if (exact >= 0) {
    don[0] = set[exact]; w[0] = 1.0;
    return 1;
  }
  real sum = 0.0;
  for (int k = 0; k < ns; k++) sum += 1.0 / d2[k];
  for (int k = 0; k < ns; k++) { don[k] = set[k]; w[k] = (1.0 / d2[k]) / sum; }
  return ns;
}

int or_assemble(or_case* c, int wrule, int overlap, int* nrec_out) {
  *nrec_out = 0;
  if (c->dim != 2) return -6;
  int ncell = c->ncell;
  int maxside = 0;
  for (int b = 0; b < c->nblock; b++) {
    if (c->blk[b].ni + 1 > maxside) maxside = c->blk[b].ni + 1;
    if (c->blk[b].nj + 1 > maxside) maxside = c->blk[b].nj + 1;
  }
  real* bx = (real*)malloc(sizeof(real) * maxside);
  real* by = (real*)malloc(sizeof(real) * maxside);
  /* 1. node classes: inactive inside another zone's body, or where another
        zone has a cell containing the node (its lowest such cell lying at
        least overlap + 3 layers inside that zone's overset sides) and a
        nearer wall (ties: the higher zone) */
  const int cut = overlap + 3;
  int nnode = 0;
  for (int b = 0; b < c->nblock; b++) nnode += (c->blk[b].ni + 1) * (c->blk[b].nj + 1);
  int8_t* inact = (int8_t*)calloc(nnode > 0 ? nnode : 1, 1);
  /* every node is classified on its own (OpenMP over the rows of a block,
     each thread with its own wall-outline buffers) */
  for (int b = 0; b < c->nblock; b++) {
    const blk_t* B = &c->blk[b];
#pragma omp parallel
    {
      real* tx = (real*)malloc(sizeof(real) * maxside);
      real* ty_ = (real*)malloc(sizeof(real) * maxside);
#pragma omp for schedule(dynamic, 1)
      for (int j = 0; j <= B->nj; j++)
        for (int i = 0; i <= B->ni; i++) {
          real px = node_x(c, b, i, j), py = node_y(c, b, i, j);
          int off = inside_body(c, b, px, py, tx, ty_);
          real da = wall_dist2(c, b, px, py, tx, ty_);
          for (int z = 0; z < c->nblock && !off; z++) {
            if (z == b) continue;
            int m = containing_cell(c, z, px, py, NULL);
            if (m < 0 || overset_depth(c, m) < cut) continue;
            real dz = wall_dist2(c, z, px, py, tx, ty_);
            if (dz < da || (dz == da && z > b)) off = 1;
          }
          inact[c->node0[b] + i + (B->ni + 1) * j] = (int8_t)off;
        }
      free(tx);
      free(ty_);
    }
  }
  /* 2. cell classes: field (all nodes active), hole (none), boundary */
  int8_t* cls = (int8_t*)malloc(ncell > 0 ? ncell : 1);
  for (int n = 0; n < ncell; n++) {
    int b = c->cblk[n], i = c->ci[n], j = c->cj[n], ni1 = c->blk[b].ni + 1, o = c->node0[b];
    int k = inact[o + i + ni1 * j] + inact[o + i + 1 + ni1 * j] + inact[o + i + 1 + ni1 * (j + 1)] +
            inact[o + i + ni1 * (j + 1)];
    cls[n] = (k == 0) ? OR_FIELD : (k == 4) ? OR_HOLE : OR_RECEPTOR;
  }
  /* 3. receptors: boundary cells, one buffer layer of field cells beside a
        boundary or hole cell, and `overlap` layers beside an overset side */
  int8_t* ty = (int8_t*)malloc(ncell > 0 ? ncell : 1);
  for (int n = 0; n < ncell; n++) {
    ty[n] = cls[n];
    if (cls[n] != OR_FIELD) continue;
    for (int dir = 0; dir < 2; dir++)
      for (int sd = -1; sd <= 1; sd += 2) {
        int m = index_nb(c, n, dir, sd);
        if (m >= 0 && cls[m] != OR_FIELD) ty[n] = OR_RECEPTOR;
      }
    const blk_t* B = &c->blk[c->cblk[n]];
    int i = c->ci[n], j = c->cj[n];
    if ((B->bc[0] == OR_NONE && i < overlap) || (B->bc[1] == OR_NONE && i >= B->ni - overlap) ||
        (B->bc[2] == OR_NONE && j < overlap) || (B->bc[3] == OR_NONE && j >= B->nj - overlap))
      ty[n] = OR_RECEPTOR;
  }
  /* 4. donors (Sec. 3.2) of the receptors, then of the cells that were
        holes and are field now (filled once, at the start of the step) */
  int nrec = 0, nref = 0;
  for (int n = 0; n < ncell; n++) {
    nrec += (ty[n] == OR_RECEPTOR);
    nref += (c->type[n] == OR_HOLE && ty[n] == OR_FIELD);
  }
  int nrow = nrec + nref;
  int* rec = (int*)malloc(sizeof(int) * (nrow > 0 ? nrow : 1));
  int* ptr = (int*)malloc(sizeof(int) * (nrow + 1));
  int* don = (int*)malloc(sizeof(int) * (5 * nrow > 0 ? 5 * nrow : 1));
  real* w = (real*)malloc(sizeof(real) * (5 * nrow > 0 ? 5 * nrow : 1));
  /* refill cells take donors among the cells that were not holes, so that
     they can be filled before the receptors (which may use them) */
  int8_t* tyr = (int8_t*)malloc(ncell > 0 ? ncell : 1);
  for (int n = 0; n < ncell; n++) tyr[n] = (c->type[n] == OR_HOLE && ty[n] == OR_FIELD) ? OR_HOLE : ty[n];
  int r = 0, nd = 0, rc = 0;
  ptr[0] = 0;
  for (int pass = 0; pass < 2 && !rc; pass++)
    for (int n = 0; n < ncell && !rc; n++) {
      int want = (pass == 0) ? ty[n] == OR_RECEPTOR : (c->type[n] == OR_HOLE && ty[n] == OR_FIELD);
      if (!want) continue;
      int k = donors_of(c, (pass == 0) ? ty : tyr, n, wrule, don + nd, w + nd);
      if (k < 0) { rc = -5; break; }
      rec[r] = n;
      nd += k;
      r++;
      ptr[r] = nd;
    }
  if (!rc) {
    memcpy(c->type, ty, ncell);
    or_set_overset(c, nrec, rec, ptr, don, w);
    /* the refill rows follow the receptors in the same table */
    free(c->rec); free(c->dptr); free(c->don); free(c->dw);
    c->rec = rec; c->dptr = ptr; c->don = don; c->dw = w;
    rec = NULL; ptr = NULL; don = NULL; w = NULL;
    c->nref = nref;
    *nrec_out = nrec;
  }
  free(bx); free(by); free(inact); free(cls); free(ty); free(tyr); free(rec); free(ptr); free(don); free(w);
  return rc;
}
