// Device-side data layout and math of libugks (gfx950).
//
// Geometry lives in struct-of-arrays device buffers owned by the context; a
// Dev value (plain pointers and sizes) is passed to every kernel by value.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ugks {

constexpr double kPi = 3.14159265358979323846;

// neighbour codes in the per-cell table nb[cell][4] (slots: i-low, i-high,
// j-low, j-high); >= 0 is a non-hole cell of the same block
constexpr int kNbFar = -1;    // far-field ghost: Maxwellian of W_inf
constexpr int kNbCopy = -2;   // zero-gradient ghost: the cell itself
constexpr int kNbWall = -3;   // isothermal wall
constexpr int kNbMiss = -4;   // hole, overset fringe or no face

// face record (double) written by the face-equilibrium kernels
enum : int {
  R_RHO = 0, R_UX, R_UY, R_LAM, R_QX, R_QY,
  R_HN,        // rho (lam/pi)^(D/2)
  R_SH,        // 4 (1-Pr) lam^2 / (5 rho)
  R_AX = 8,    // slope coefficients along x (4)
  R_AY = 12,   // along y (4)
  R_AT = 16,   // time coefficients A (4)
  R_T1 = 20,   // q1..q5 / dt_s (5)
  R_ACT = 25,  // 1 if the face carries flux
  R_RHOW,      // wall density
  R_LAMW,      // 1/(2 RT_w)
  R_HWN,       // (lam_w/pi)^(D/2)
  R_VWX, R_VWY,
  R_SGN,       // +1: face normal points into the wall
  R_RT = 32,   // 1/(2 lam)
  R_SQX, R_SQY,  // R_SH * q
  R_SX, R_SY,  // moment shift of the face (mean velocity of its two sides)
  // 2D: the interface distribution as polynomials in c = v - U (below)
  R_PH = 40,   // cubic Q_h: c00 c01 c02 c03 c10 c11 c12 c20 c21 c30 (10)
  R_LB = 50,   // linear part of Q_b: l0 lx ly (3)
  R_KB = 53,   // Q_b = R_KB Q_h + L_b
  NREC = 56
};

// cubic polynomials in two variables: c[i][j] multiplies X^i Y^j, i + j <= 3
struct Poly3 {
  double c[4][4];
};
__device__ inline Poly3 poly_lin(double a0, double ax, double ay) {
  Poly3 p = {};
  p.c[0][0] = a0; p.c[1][0] = ax; p.c[0][1] = ay;
  return p;
}
__device__ inline Poly3 poly_axpy(double s, const Poly3& a, const Poly3& b) {  // s a + b
  Poly3 p;
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) p.c[i][j] = s * a.c[i][j] + b.c[i][j];
  return p;
}
__device__ inline Poly3 poly_mul(const Poly3& a, const Poly3& b) {  // degrees add up to at most 3 here
  Poly3 p = {};
  for (int i = 0; i < 4; ++i)
    for (int j = 0; i + j < 4; ++j)
      for (int k = 0; i + k < 4; ++k)
        for (int l = 0; j + l < 4 && i + k + j + l < 4; ++l) p.c[i + k][j + l] += a.c[i][j] * b.c[k][l];
  return p;
}

// derived fields of a face record used per velocity.  In 2D the interface
// distribution of Eq. fullSolution integrated over dt_s (face state U, lam,
// q; slopes a_x, a_y; time coefficient A; integrals q1..q5; face grid
// velocity Uf, w = v - Uf) is
//   I_h = q1 f_h + q2 w.grad f_h + exp(-lam |c|^2) Q_h(c),
//   I_b = q1 f_b + q2 w.grad f_b + exp(-lam |c|^2) (K_b Q_h(c) + L_b(c)),
// c = v - U: the Maxwellian's prefactor, the Shakhov factor, (w.a) and A.psi
// collected into one cubic Q_h and a linear L_b, once per face instead of
// once per velocity
__device__ inline void record_derived(double* r, int dim, int nxi, double ufx, double ufy) {
  r[R_RT] = 0.5 / r[R_LAM];
  r[R_SQX] = r[R_SH] * r[R_QX];
  r[R_SQY] = r[R_SH] * r[R_QY];
  if (dim != 2) return;
  const double lam = r[R_LAM], rt = r[R_RT], hn = r[R_HN], ux = r[R_UX], uy = r[R_UY];
  const double sqx = r[R_SQX], sqy = r[R_SQY];
  const double* ax = r + R_AX;
  const double* ay = r + R_AY;
  const double* at = r + R_AT;
  const double* t = r + R_T1;
  const double dx = ux - ufx, dy = uy - ufy;  // w = c + (U - Uf)
  const Poly3 X = poly_lin(0.0, 1.0, 0.0), Y = poly_lin(0.0, 0.0, 1.0);
  const Poly3 one = poly_lin(1.0, 0.0, 0.0);
  const Poly3 s = poly_lin(0.0, sqx, sqy);                                   // c.(Shakhov q)
  const Poly3 c2 = poly_axpy(1.0, poly_mul(X, X), poly_mul(Y, Y));
  // 1 + s (2 lam |c|^2 - 2 - D): Maxwellian plus its Shakhov part for h
  const Poly3 shk = poly_axpy(1.0, one, poly_mul(s, poly_axpy(2.0 * lam, c2, poly_lin(-2.0 - dim, 0.0, 0.0))));
  // energy factor of (a.psi) for h: (|v|^2 + nxi rt) / 2
  const Poly3 vx = poly_lin(ux, 1.0, 0.0), vy = poly_lin(uy, 0.0, 1.0);
  const Poly3 eh = poly_axpy(0.5, poly_axpy(1.0, poly_mul(vx, vx), poly_mul(vy, vy)),
                             poly_lin(0.5 * nxi * rt, 0.0, 0.0));
  const Poly3 pax = poly_lin(ax[0] + ax[1] * ux + ax[2] * uy, ax[1], ax[2]);
  const Poly3 pay = poly_lin(ay[0] + ay[1] * ux + ay[2] * uy, ay[1], ay[2]);
  const Poly3 pat = poly_lin(at[0] + at[1] * ux + at[2] * uy, at[1], at[2]);
  const Poly3 wx = poly_lin(dx, 1.0, 0.0), wy = poly_lin(dy, 0.0, 1.0);
  const Poly3 wah = poly_axpy(1.0, poly_mul(wx, poly_axpy(ax[3], eh, pax)), poly_mul(wy, poly_axpy(ay[3], eh, pay)));
  const Poly3 ath = poly_axpy(at[3], eh, pat);
  const Poly3 ph = poly_axpy(t[2], shk, poly_axpy(t[3], wah, poly_axpy(t[4], ath, Poly3{})));
  const double q[10] = {ph.c[0][0], ph.c[0][1], ph.c[0][2], ph.c[0][3], ph.c[1][0],
                        ph.c[1][1], ph.c[1][2], ph.c[2][0], ph.c[2][1], ph.c[3][0]};
  for (int m = 0; m < 10; ++m) r[R_PH + m] = hn * q[m];
  // Q_b = nxi rt hn (P_h + 2 q3 s + rt (q4 (w_x a_x3 + w_y a_y3) + q5 A_3))
  const double kb = nxi * rt, hb = hn * kb;
  r[R_KB] = kb;
  r[R_LB] = hb * rt * (t[3] * (ax[3] * dx + ay[3] * dy) + t[4] * at[3]);
  r[R_LB + 1] = hb * (2.0 * t[2] * sqx + rt * t[3] * ax[3]);
  r[R_LB + 2] = hb * (2.0 * t[2] * sqy + rt * t[3] * ay[3]);
}

// packed per-cell table of the march kernels (one double per entry; kinds
// and indices as int32 in the low word, high word zero, so that a lane read
// of the low word gives the integer): kind, neighbour codes per slot,
// J^{-T}, face area per slot (0 without a face), 1/|Omega|, face id per slot
// (-1 none)
enum : int { kCpType = 0, kCpNb = 1, kCpG = 5, kCpS = 9, kCpIvol = 13, kCpFace = 14, kCpN = 20 };
// an int32 entry of the packed march tables (low word, high word zero) and
// its read-back
inline double tab_int_entry(int v) {
  const unsigned long long u = (unsigned long long)(unsigned int)v;
  double d;
  __builtin_memcpy(&d, &u, sizeof d);
  return d;
}
__host__ __device__ __forceinline__ int tab_int(double v) {
  unsigned long long u;
  __builtin_memcpy(&u, &v, sizeof u);
  return (int)(unsigned int)(u & 0xffffffffull);
}
// packed per-face table: unit normal, area, grid velocity, offsets from the
// centroids of the low and high cells to the face centre (zero on a ghost or
// wall side), low and high cell or ghost code, 1 if the face carries flux
// (the last three int32 entries, read with tab_int)
enum : int { kFpN0 = 0, kFpS = 2, kFpU = 3, kFpDL = 5, kFpDR = 7, kFpL = 9, kFpR = 10, kFpAct = 11, kFpN = 12 };

// wall table entry (double; the face id as an int32 entry): face id, area,
// sign turning the face normal into the normal pointing into the wall, that
// inward normal, face centre relative to the block's moved rotation centre
enum : int { kWtFace = 0, kWtS, kWtSgn, kWtNx, kWtNy, kWtRx, kWtRy, kWtN = 8 };

// per-cell record (double): state of the Shakhov source, the micro LU-SGS
// diagonal base 1/dt' + 1/dt + 1/(2 tau) and, per slot s, the face
// coefficients (A, B, C) with S/(2|Omega|) * w.n_out = A vx + B vy - C
enum : int {
  C_RHO = 0, C_UX, C_UY, C_LAM, C_QX, C_QY, C_HN, C_SH, C_ITAU, C_GEO = 10, C_D0 = 22, C_FLD = 23, NCREC = 24
};

// per-cell moment record about a shift s: s(2), m0, m1(2), m2, P(3), m3(2)
enum : int {
  M_SX = 0, M_SY, M_M0, M_M1X, M_M1Y, M_M2, M_PXX, M_PXY, M_PYY, M_M3X, M_M3Y, NMREC = 11
};

struct Dev {
  int dim, nxi, nw, nv, nvx, nvy, ncell, nface, nblock;
  double pr, omega, mu_ref, rt_ref;
  double winf[4];
  const double* vx;     // [nv]
  const double* vy;     // [nv]
  const double* wk;     // [nv] velocity weights
  const double* vol;    // [ncell]
  const double* G;      // [ncell][4] J^{-T}
  const double* cdx;    // [ncell][8] face centre - centroid per slot
  const double* dtp;    // [ncell]
  const int8_t* type;   // [ncell]
  const int* nb;        // [ncell][4]
  const int* cf;        // [ncell][4] face per slot or -1
  const int* fcell;     // [nface][2] L, R (cell or ghost code)
  const double* fgeo;   // [nface][8] nx, ny, S, ux, uy, vwx, vwy, rtw
  const int8_t* fact;   // [nface] face adjacent to a field cell
  const void* finf_h;   // [nv] storage type
  const void* finf_b;
  const double* mgeo;   // [ncell][12] per slot (A, B, C) of the micro sweep
  // packed per-cell and per-face tables of the march kernels (layouts
  // kCp* and kFp* below), rebuilt with the geometry and the cell kinds
  const double* cplan;  // [ncell][kCpN]
  const double* fplan;  // [nface][kFpN]
  // launch shapes (read by the host launchers only; results do not depend
  // on them): widest velocity chunk of the micro sweep, core rows per
  // workgroup of the face-equilibrium and flux march kernels
  int kc_max = 16, rg_eq = 8, rg_flux = 8;
  // device status word of the context (bits kStatus*), set by the kernels
  // that detect a failure and read by the host at a synchronisation
  unsigned* status = nullptr;
  // bound of the micro sweep's wait for its neighbour wavefronts (sleeps)
  int micro_spin = 1 << 20;
};

// bits of the device status word
constexpr unsigned kStatusWait = 1u;     // a sweep's neighbour wait ran out
constexpr unsigned kStatusNonPhys = 2u;  // Step 7 produced rho <= 0, T <= 0 or a non-finite W

// sets bits of the status word (one vector atomic per calling lane)
__device__ __forceinline__ void raise_status(unsigned* st, unsigned bits) {
  if (st) __hip_atomic_fetch_or(st, bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ------------------------------------------------------------------------
// gas relations
// ------------------------------------------------------------------------
__device__ __host__ inline void prim_of(const Dev& g, const double* W, double& rho, double& ux,
                                        double& uy, double& lam) {
  rho = W[0];
  ux = W[1] / rho;
  uy = (g.dim == 2) ? W[2] / rho : 0.0;
  double e = W[g.dim + 1] - 0.5 * rho * (ux * ux + uy * uy);
  lam = 0.25 * (double)(g.dim + g.nxi) * rho / e;
}

// positive density and internal energy
__device__ __host__ __forceinline__ bool physical_state(int dim, const double* W) {
  if (!(W[0] > 0.0)) return false;
  double ke = W[1] * W[1] + ((dim == 2) ? W[2] * W[2] : 0.0);
  return W[dim + 1] - 0.5 * ke / W[0] > 0.0;
}

// (the gas relations below are templates on the scalar type R: double in
// the solver, a forward-mode dual number in the adjoint's local Jacobians)
template <class R>
__device__ inline R inv_tau_of(const Dev& g, R rho, R lam) {
  if (g.mu_ref <= 0.0) return R(0.0);
  R rt = 0.5 / lam;
  R mu = g.mu_ref * pow(rt / g.rt_ref, g.omega);
  return rho * rt / mu;
}

// time integrals q1..q5 over [0, dts] of the interface-solution coefficients;
// Taylor series below x = 1 (m <= 24), closed forms above
template <class R>
__device__ inline void time_integrals(double dts, R itau, R* q) {
  R x = dts * itau;
  if (x < 1.0) {
    R a1 = 0.0, a2 = 0.0, a3 = 0.0, a4 = 0.0, a5 = 0.0;
    R p = 1.0;  // x^(m-1)
    R pp = 0.0; // x^(m-2)
    double fac = 1.0;
    for (int m = 1; m <= 24; ++m) {
      fac *= (double)m;
      double s = (m & 1) ? 1.0 : -1.0;  // (-1)^(m+1)
      a1 += s * p / fac;
      if (m >= 2) {
        a3 -= s * p / fac;
        a2 += s * (double)(m - 1) * pp / fac;
      }
      if (m >= 3) {
        a4 -= s * (double)(m - 2) * pp / fac;
        a5 += s * pp / fac;
      }
      pp = (m == 1) ? 1.0 : pp * x;
      p *= x;
    }
    q[0] = dts * a1;
    q[1] = dts * dts * a2;
    q[2] = dts * a3;
    q[3] = dts * dts * a4;
    q[4] = dts * dts * a5;
  } else {
    R tau = 1.0 / itau;
    R e = exp(-x);
    q[0] = tau * (1.0 - e);
    q[1] = tau * tau * ((1.0 + x) * e - 1.0);
    q[2] = dts - q[0];
    q[3] = tau * tau * (2.0 - x - (2.0 + x) * e);
    q[4] = tau * tau * (0.5 * x * x - x + 1.0 - e);
  }
}

// closed-form inverse of the Maxwellian moment matrix: a with <psi psi^T> a = d
// (gas-kinetic micro-slope formulas; K' = N_xi internal components)
template <class R>
__device__ inline void slope_inverse(int dim, R U, R V, R lam, const R* d, R* a) {
  if (dim == 2) {
    const double K = 1.0;
    R e2 = U * U + V * V + (K + 2.0) / (2.0 * lam);
    R r4 = 2.0 * d[3] - e2 * d[0];
    R r3 = d[2] - V * d[0];
    R r2 = d[1] - U * d[0];
    a[3] = 4.0 * lam * lam / (K + 2.0) * (r4 - 2.0 * U * r2 - 2.0 * V * r3);
    a[2] = 2.0 * lam * r3 - V * a[3];
    a[1] = 2.0 * lam * r2 - U * a[3];
    a[0] = d[0] - U * a[1] - V * a[2] - 0.5 * a[3] * e2;
  } else {
    const double K = 2.0;
    R e2 = U * U + (K + 1.0) / (2.0 * lam);
    R r3 = 2.0 * d[2] - e2 * d[0];
    R r2 = d[1] - U * d[0];
    a[2] = 4.0 * lam * lam / (K + 1.0) * (r3 - 2.0 * U * r2);
    a[1] = 2.0 * lam * r2 - U * a[2];
    a[0] = d[0] - U * a[1] - 0.5 * a[2] * e2;
  }
}

// <psi v_dir (a . psi)> under the normalised Maxwellian (mean U, V; 1/(2 lam))
template <class R>
__device__ inline void psi_v_apsi(int dim, int dir, R U, R V, R lam, const R* a, R* out) {
  R th = 0.5 / lam;
  R mu[7], mv[7];
  mu[0] = 1.0; mu[1] = U;
  mv[0] = 1.0; mv[1] = V;
  for (int n = 1; n < 6; ++n) {
    mu[n + 1] = U * mu[n] + n * th * mu[n - 1];
    mv[n + 1] = V * mv[n] + n * th * mv[n - 1];
  }
  if (dim == 1) {
    R x1 = 2.0 * th, x2 = 8.0 * th * th;  // <xi^2>, <xi^4> for 2 components
    R uE = 0.5 * (mu[3] + mu[1] * x1);
    R u2E = 0.5 * (mu[4] + mu[2] * x1);
    R uE2 = 0.25 * (mu[5] + 2.0 * mu[3] * x1 + mu[1] * x2);
    out[0] = a[0] * mu[1] + a[1] * mu[2] + a[2] * uE;
    out[1] = a[0] * mu[2] + a[1] * mu[3] + a[2] * u2E;
    out[2] = a[0] * uE + a[1] * u2E + a[2] * uE2;
    return;
  }
  R x1 = th, x2 = 3.0 * th * th;  // one internal component
  if (dir == 1) {  // swap roles of the two axes
    for (int n = 0; n < 7; ++n) { R t = mu[n]; mu[n] = mv[n]; mv[n] = t; }
  }
  // moments with w the chosen axis (mu) and z the other (mv)
  R wE = 0.5 * (mu[3] + mu[1] * mv[2] + mu[1] * x1);
  R w2E = 0.5 * (mu[4] + mu[2] * mv[2] + mu[2] * x1);
  R wzE = 0.5 * (mu[3] * mv[1] + mu[1] * mv[3] + mu[1] * mv[1] * x1);
  R wE2 = 0.25 * (mu[5] + mu[1] * mv[4] + mu[1] * x2 + 2.0 * mu[3] * mv[2] +
                  2.0 * mu[3] * x1 + 2.0 * mu[1] * mv[2] * x1);
  // coefficient along the chosen axis and along the other
  R aw = (dir == 0) ? a[1] : a[2];
  R az = (dir == 0) ? a[2] : a[1];
  R o0 = a[0] * mu[1] + aw * mu[2] + az * mu[1] * mv[1] + a[3] * wE;
  R ow = a[0] * mu[2] + aw * mu[3] + az * mu[2] * mv[1] + a[3] * w2E;
  R oz = a[0] * mu[1] * mv[1] + aw * mu[2] * mv[1] + az * mu[1] * mv[2] + a[3] * wzE;
  R oE = a[0] * wE + aw * w2E + az * wzE + a[3] * wE2;
  out[0] = o0;
  out[1] = (dir == 0) ? ow : oz;
  out[2] = (dir == 0) ? oz : ow;
  out[3] = oE;
}

// equilibrium expansion coefficients of a face state: slopes a_d from the
// gradient dW[d][nw] and time coefficient A from the compatibility condition
// with the relative velocity w = v - U_f
template <class R>
__device__ inline void expansion(int dim, R rho, R U, R V, R lam, R ufx, R ufy, const R* dW, R* ax, R* ay,
                                 R* At) {
  int nw = dim + 2;
  R d[4];
  for (int m = 0; m < nw; ++m) d[m] = dW[m] / rho;
  slope_inverse(dim, U, V, lam, d, ax);
  R b[4] = {0.0, 0.0, 0.0, 0.0};
  R t[4];
  psi_v_apsi(dim, 0, U, V, lam, ax, t);
  for (int m = 0; m < nw; ++m) b[m] = -t[m] + ufx * d[m];
  if (dim == 2) {
    for (int m = 0; m < nw; ++m) d[m] = dW[nw + m] / rho;
    slope_inverse(dim, U, V, lam, d, ay);
    psi_v_apsi(dim, 1, U, V, lam, ay, t);
    for (int m = 0; m < nw; ++m) b[m] += -t[m] + ufy * d[m];
  } else {
    for (int m = 0; m < 4; ++m) ay[m] = R(0.0);
  }
  slope_inverse(dim, U, V, lam, b, At);
  if (dim == 1) { ax[3] = R(0.0); At[3] = R(0.0); }
}

// Workgroup barrier that orders LDS accesses only.  The LU-SGS sweeps hand
// values between threads through LDS; their global stores are read back
// only by the thread that wrote them, so the barrier need not wait for them
// (the full __syncthreads fence would drain every outstanding global load
// and store each hyperplane, defeating the prefetch).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// ------------------------------------------------------------------------
// wavefront reduction (64 lanes)
// ------------------------------------------------------------------------
// lane permutation of a double through DPP (both 32-bit halves)
template <int CTRL>
__device__ __forceinline__ double dpp_perm(double v) {
  int lo = __double2loint(v), hi = __double2hiint(v);
  // every control used here (quad permutes, row mirrors) reads a lane of
  // the same row, so no lane keeps an old value: the plain DPP move needs
  // no zeroed destination
  lo = __builtin_amdgcn_mov_dpp(lo, CTRL, 0xF, 0xF, false);
  hi = __builtin_amdgcn_mov_dpp(hi, CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double lane_read(double v, int l) {
  int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}

// sum over the 64 lanes, returned to every lane: pairs, quads, half rows
// and rows of 16 through DPP, then the four row sums in a fixed order
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_perm<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_perm<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_perm<0x141>(v);  // row_half_mirror
  v += dpp_perm<0x140>(v);  // row_mirror
  return (lane_read(v, 0) + lane_read(v, 16)) + (lane_read(v, 32) + lane_read(v, 48));
}

// exchange of doubles between lane groups (gfx950 permlane swaps): W = 32
// swaps lanes 32-63 of x with lanes 0-31 of y; W = 16 swaps lanes 16-31 and
// 48-63 of x with lanes 0-15 and 32-47 of y
template <int W>
__device__ __forceinline__ void lane_swap(double& x, double& y) {
  const unsigned xl = (unsigned)__double2loint(x), xh = (unsigned)__double2hiint(x);
  const unsigned yl = (unsigned)__double2loint(y), yh = (unsigned)__double2hiint(y);
  if constexpr (W == 32) {
    const auto lo = __builtin_amdgcn_permlane32_swap(xl, yl, false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap(xh, yh, false, false);
    x = __hiloint2double((int)hi[0], (int)lo[0]);
    y = __hiloint2double((int)hi[1], (int)lo[1]);
  } else {
    const auto lo = __builtin_amdgcn_permlane16_swap(xl, yl, false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap(xh, yh, false, false);
    x = __hiloint2double((int)hi[0], (int)lo[0]);
    y = __hiloint2double((int)hi[1], (int)lo[1]);
  }
}

// one reduce-scatter stage over lane bit B: n values in, n/2 out (n >= 2),
// the lanes with bit B set keep the upper half of the indices; with n = 1 a
// butterfly (both partners get the pair sum)
template <int B>
__device__ __forceinline__ void rs_stage(double* v, int n, int lane) {
  const bool up = (lane >> B) & 1;
  if (n == 1) {
    if constexpr (B == 5 || B == 4) {
      double a = v[0], b = v[0];
      lane_swap<(B == 5) ? 32 : 16>(a, b);
      v[0] = a + b;
    } else {
      constexpr int CTRL = (B == 3) ? 0x140 : (B == 2) ? 0x141 : (B == 1) ? 0x4E : 0xB1;
      v[0] = v[0] + dpp_perm<CTRL>(v[0]);
    }
    return;
  }
  const int hn = n / 2;
  for (int i = 0; i < hn; ++i) {
    if constexpr (B == 5 || B == 4) {
      double a = v[i], b = v[i + hn];
      lane_swap<(B == 5) ? 32 : 16>(a, b);
      v[i] = a + b;
    } else {
      constexpr int CTRL = (B == 3) ? 0x140 : (B == 2) ? 0x141 : (B == 1) ? 0x4E : 0xB1;
      const double send = up ? v[i] : v[i + hn];
      const double keep = up ? v[i + hn] : v[i];
      v[i] = keep + dpp_perm<CTRL>(send);
    }
  }
}

// Sums over the 64 lanes of V values at once (V = 1, 2, 4, 8 or 16), far
// cheaper than V separate reductions: each stage halves the values a lane
// carries.  On return v[0] of lane l holds the total of value l >> (6 - log2 V)
// (every lane of that group holds the same, bit-identical total; the order of
// the additions is fixed).
template <int V>
__device__ __forceinline__ void multi_sum(double* v, int lane) {
  static_assert(V == 1 || V == 2 || V == 4 || V == 8 || V == 16, "V");
  int n = V;
  rs_stage<5>(v, n, lane); n = (n > 1) ? n / 2 : 1;
  rs_stage<4>(v, n, lane); n = (n > 1) ? n / 2 : 1;
  rs_stage<3>(v, n, lane); n = (n > 1) ? n / 2 : 1;
  rs_stage<2>(v, n, lane); n = (n > 1) ? n / 2 : 1;
  rs_stage<1>(v, n, lane); n = (n > 1) ? n / 2 : 1;
  rs_stage<0>(v, n, lane);
}

template <class T>
__device__ inline double ld(const T* p, size_t i) { return (double)p[i]; }

}  // namespace ugks
