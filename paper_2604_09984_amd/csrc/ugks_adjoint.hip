// Hand-written reverse mode (vector-Jacobian products) of the dual-time
// pseudo-iteration (Sec. 2.2, Steps 3-7) and of Steps 1-2, FP64 storage.
//
// Each kernel is the transpose of one stage of the solver, applied to
// cotangents ("bars") at a forward state that the host recomputes first
// (checkpointed recomputation): the stages run backwards, Step 7 and the
// heat flux first, then the micro LU-SGS sweeps (transposed sweeps in
// reversed hyperplane order), the macro LU-SGS (reverse of the two nonlinear
// sweeps), the UGKS interface flux (per face, threads over velocities) and
// the overset interpolation.  Small dense per-face maps (the equilibrium
// expansion coefficients and the time integrals of Eq. fullSolution) are
// differentiated in forward mode, one input direction per lane, and the
// resulting Jacobian columns are contracted with the cotangent in the same
// lanes.  Contributions that several items (faces, cells, donor rows) add
// to one cell run over a write-disjoint colouring of the items, one launch
// per colour, and contributions of a cell to its own faces are gathered per
// face: every sum has a fixed order and the results are bitwise
// reproducible.
//
// Differentiated quantities: the distribution (h, b), W, q and the dual-time
// sources of a step; the face grid velocity U_f (Eq. BGK, w = v - U), the
// wall velocity and the wall temperature (Eq. maxWalldes) per face.  Frozen:
// node positions, cell kinds and donor tables, dt, dt_s and the virtual
// steps dt'.  At the kinks of the method (limiter switch, upwind sign,
// positivity fallbacks, |.| in the spectral radius) the derivative of the
// branch the forward pass took is used.
#include "ugks_adjoint.h"
#include "ugks_dev.h"

namespace ugks {

// The reverse-mode entry points accept 2D cases only (checked on the host);
// compile-time sizes keep the small per-face and per-cell arrays in registers.
constexpr int kD = 2, kNxi = 1, kNw = 4;


// ------------------------------------------------------------------------
// forward-mode scalar (value and one directional derivative)
// ------------------------------------------------------------------------
struct Fwd {
  double v, d;
  Fwd() = default;
  __device__ constexpr Fwd(double x) : v(x), d(0.0) {}
  __device__ constexpr Fwd(double x, double t) : v(x), d(t) {}
};
__device__ inline Fwd operator+(Fwd a, Fwd b) { return Fwd(a.v + b.v, a.d + b.d); }
__device__ inline Fwd operator-(Fwd a, Fwd b) { return Fwd(a.v - b.v, a.d - b.d); }
__device__ inline Fwd operator-(Fwd a) { return Fwd(-a.v, -a.d); }
__device__ inline Fwd operator*(Fwd a, Fwd b) { return Fwd(a.v * b.v, a.d * b.v + a.v * b.d); }
__device__ inline Fwd operator/(Fwd a, Fwd b) {
  double q = a.v / b.v;
  return Fwd(q, (a.d - q * b.d) / b.v);
}
__device__ inline Fwd& operator+=(Fwd& a, Fwd b) { a = a + b; return a; }
__device__ inline Fwd& operator-=(Fwd& a, Fwd b) { a = a - b; return a; }
__device__ inline Fwd& operator*=(Fwd& a, Fwd b) { a = a * b; return a; }
__device__ inline bool operator<(Fwd a, Fwd b) { return a.v < b.v; }
__device__ inline bool operator>(Fwd a, Fwd b) { return a.v > b.v; }
__device__ inline Fwd exp(Fwd a) { double e = ::exp(a.v); return Fwd(e, e * a.d); }
__device__ inline Fwd pow(Fwd a, double b) {
  double p = ::pow(a.v, b);
  return Fwd(p, b * ::pow(a.v, b - 1.0) * a.d);
}
// the double overloads stay visible beside the ones above
using ::exp;
using ::pow;

// ------------------------------------------------------------------------
// small helpers
// ------------------------------------------------------------------------
// scatter update.  The kernels that scatter run over one colour of a
// write-disjoint colouring of their items at a time (faces, cells or donor
// rows), so no two threads of a launch update one address, and one thread's
// updates of an address take effect in program order: every sum is formed
// in an order fixed by the colouring, independent of scheduling.  The
// update is issued as an atomic add without return only so that the thread
// does not wait for the old value.
__device__ __forceinline__ void acc_add(double* p, double v) {
  if (v != 0.0) unsafeAtomicAdd(p, v);
}

// (v - U).n with the same rounding as the solver's upwind decision
__device__ __forceinline__ double wn_exact(double vx, double vy, double ux, double uy, double nx, double ny) {
#pragma clang fp contract(off)
  double a = (vx - ux) * nx;
  double b = (vy - uy) * ny;
  return a + b;
}

// reverse of (rho, U, lam) = prim(W): W_bar += J^T (rho_bar, u_bar, lam_bar)
__device__ inline void prim_rev(int dim, int nxi, const double* W, double rb, double uxb, double uyb, double lb,
                                double* Wb) {
  double rho = W[0];
  double ux = W[1] / rho, uy = (dim == 2) ? W[2] / rho : 0.0;
  double e = W[dim + 1] - 0.5 * rho * (ux * ux + uy * uy);
  double lam = 0.25 * (double)(dim + nxi) * rho / e;
  // lam = K rho / (4 e): d/drho (explicit) = lam/rho, d/de = -lam/e
  double eb = -lb * lam / e;
  Wb[0] += rb - uxb * ux / rho - uyb * uy / rho + lb * lam / rho + eb * 0.5 * (ux * ux + uy * uy);
  Wb[1] += uxb / rho - eb * ux;
  if (dim == 2) Wb[2] += uyb / rho - eb * uy;
  Wb[dim + 1] += eb;
}

__device__ inline void prim_d(int dim, int nxi, const double* W, double& rho, double& ux, double& uy, double& lam) {
  rho = W[0];
  ux = W[1] / rho;
  uy = (dim == 2) ? W[2] / rho : 0.0;
  double e = W[dim + 1] - 0.5 * rho * (ux * ux + uy * uy);
  lam = 0.25 * (double)(dim + nxi) * rho / e;
}

// d(1/tau)/d(rho, lam) at (rho, lam)
__device__ inline void itau_partials(const Dev& g, double rho, double lam, double& dr, double& dl) {
  double it = inv_tau_of(g, rho, lam);
  dr = it / rho;
  dl = -it * (1.0 - g.omega) / lam;
}

// Reverse of the reduced Shakhov equilibrium (Sec. 2.1) at one velocity:
// (rho, U, lam, q) -> H, B (Maxwellian), Hp = H+ and Bp = B+ (the Shakhov
// corrections), given the cotangents of those four values; accumulates into
// a[0..5] = (rho, ux, uy, lam, qx, qy) bars.
__device__ inline void eq_rev(const Dev& g, double rho, double ux, double uy, double lam, double qx, double qy,
                              double vx, double vy, double Hb, double Bb, double Hpb, double Bpb, double* a) {
  const int D = kD, nxi = kNxi;
  double cx = vx - ux, cy = (D == 2) ? vy - uy : 0.0;
  double c2 = cx * cx + cy * cy;
  double H = rho * pow(lam / kPi, 0.5 * D) * exp(-lam * c2);
  double beta = (double)nxi / (2.0 * lam);
  double sh = 4.0 * (1.0 - g.pr) * lam * lam / (5.0 * rho);
  double cq = cx * qx + cy * qy;
  double s = sh * cq;
  double P = s * (2.0 * lam * c2 - 2.0 - D), Qb = s * (2.0 * lam * c2 - D);
  double Ht = Hb + Bb * beta + Hpb * P + Bpb * Qb * beta;
  double betab = Bb * H + Bpb * Qb * H;
  double Pb = Hpb * H, Qbb = Bpb * beta * H;
  double sb = Pb * (2.0 * lam * c2 - 2.0 - D) + Qbb * (2.0 * lam * c2 - D);
  double lb = (Pb + Qbb) * s * 2.0 * c2 - betab * beta / lam;
  double c2b = (Pb + Qbb) * s * 2.0 * lam;
  double shb = sb * cq, cqb = sb * sh;
  lb += shb * 2.0 * sh / lam;
  double rb = -shb * sh / rho;
  a[4] += cqb * cx;
  if (D == 2) a[5] += cqb * cy;
  double cxb = cqb * qx, cyb = cqb * qy;
  lb += Ht * H * (0.5 * D / lam - c2);
  rb += Ht * H / rho;
  c2b += -Ht * H * lam;
  cxb += 2.0 * cx * c2b;
  cyb += 2.0 * cy * c2b;
  a[0] += rb;
  a[1] -= cxb;
  if (D == 2) a[2] -= cyb;
  a[3] += lb;
}

// heat flux q = 1/2 sum_k V_k c (|c|^2 h + b), c = v - U: per-velocity part of
// its reverse (u_bar contribution; the h, b bars are returned)
__device__ inline void heat_rev_k(int D, double w, double vx, double vy, double ux, double uy, double hv,
                                  double bv, double qxb, double qyb, double& hb, double& bb, double& uxb,
                                  double& uyb) {
  double cx = vx - ux, cy = (D == 2) ? vy - uy : 0.0;
  double c2 = cx * cx + cy * cy;
  double cqb = cx * qxb + cy * qyb;
  hb = w * 0.5 * cqb * c2;
  bb = w * 0.5 * cqb;
  double e = c2 * hv + bv;
  uxb += -0.5 * w * (qxb * (e + 2.0 * cx * cx * hv) + qyb * 2.0 * cx * cy * hv);
  if (D == 2) uyb += -0.5 * w * (qyb * (e + 2.0 * cy * cy * hv) + qxb * 2.0 * cx * cy * hv);
}

// ------------------------------------------------------------------------
// face equilibrium record and the per-velocity interface integral
// ------------------------------------------------------------------------
// expansion coefficients (a_x, a_y, A) and time integrals q1..q5 of a face
// state; inputs x = (rho, ux, uy, lam, dW[8] as the gradient layout, ufx, ufy)
constexpr int kRecIn = 14, kRecOut = 17;
template <class R>
__device__ inline void face_coeffs(const Dev& g, double dts, const R* x, R* o) {
  expansion(kD, x[0], x[1], x[2], x[3], x[12], x[13], x + 4, o, o + 4, o + 8);
  time_integrals(dts, inv_tau_of(g, x[0], x[3]), o + 12);
}

// values of the record (all lanes) and, in lane j < kRecIn, the derivatives
// of the outputs along input j
__device__ inline void face_coeffs_lanes(const Dev& g, double dts, const double* x, int lane, double* val,
                                         double* col) {
  Fwd xi[kRecIn], o[kRecOut];
  for (int j = 0; j < kRecIn; ++j) xi[j] = Fwd(x[j], (j == lane) ? 1.0 : 0.0);
  face_coeffs(g, dts, xi, o);
  for (int i = 0; i < kRecOut; ++i) { val[i] = o[i].v; col[i] = o[i].d; }
}

struct Rec {
  double rho, ux, uy, lam, qx, qy;
  double c[kRecOut];  // ax[4], ay[4], A[4], t[5]
};

// record cotangent: [0..5] rho, ux, uy, lam, qx, qy; [6..22] the kRecOut
// coefficients; [23..24] w = v - U_f (its bar is minus the U_f bar)
constexpr int kRecBar = 25;

// Interface integral of Eq. fullSolution at one velocity (Ih, Ib: the time
// integral over [0, dt_s] of the interface distribution) and its reverse
// for the cotangents Ihb, Ibb.  Per-velocity bars of the side data are
// returned; record bars are accumulated into acc[kRecBar].
template <bool ACC>
__device__ __forceinline__ void iint_rev(const Dev& g, const Rec& e, double vx, double vy, double wx, double wy,
                                         double fh, double fb, double ghx, double ghy, double gbx, double gby,
                                         double Ihb, double Ibb, double& fhb, double& fbb, double* ghb, double* gbb,
                                         double* acc, double& Ih, double& Ib) {
  const int D = kD, nxi = kNxi, E = D + 1;
  const double* ax = e.c;
  const double* ay = e.c + 4;
  const double* At = e.c + 8;
  const double* t = e.c + 12;
  double cx = vx - e.ux, cy = (D == 2) ? vy - e.uy : 0.0;
  double c2 = cx * cx + cy * cy;
  double H = e.rho * pow(e.lam / kPi, 0.5 * D) * exp(-e.lam * c2);
  double beta = (double)nxi / (2.0 * e.lam);
  double B = beta * H;
  double sh = 4.0 * (1.0 - g.pr) * e.lam * e.lam / (5.0 * e.rho);
  double s = sh * (cx * e.qx + cy * e.qy);
  double Hp = s * (2.0 * e.lam * c2 - 2.0 - D) * H;
  double Bp = s * (2.0 * e.lam * c2 - D) * beta * H;
  double v2 = vx * vx + ((D == 2) ? vy * vy : 0.0);
  double kh = 0.5 * (v2 + (double)nxi / (2.0 * e.lam)), kb = 0.5 * (v2 + (double)(nxi + 2) / (2.0 * e.lam));
  auto lin = [&](const double* a) { return a[0] + a[1] * vx + ((D == 2) ? a[2] * vy : 0.0); };
  double pax = lin(ax), pay = (D == 2) ? lin(ay) : 0.0, pat = lin(At);
  double wah = wx * (pax + ax[E] * kh) + wy * (pay + ay[E] * kh);
  double wab = wx * (pax + ax[E] * kb) + wy * (pay + ay[E] * kb);
  double Ah = pat + At[E] * kh, Ab = pat + At[E] * kb;
  double wgh = wx * ghx + wy * ghy, wgb = wx * gbx + wy * gby;
  Ih = t[0] * fh + t[1] * wgh + t[2] * (H + Hp) + t[3] * wah * H + t[4] * Ah * H;
  Ib = t[0] * fb + t[1] * wgb + t[2] * (B + Bp) + t[3] * wab * B + t[4] * Ab * B;
  // reverse
  fhb = t[0] * Ihb;
  fbb = t[0] * Ibb;
  ghb[0] = t[1] * Ihb * wx; ghb[1] = t[1] * Ihb * wy;
  gbb[0] = t[1] * Ibb * wx; gbb[1] = t[1] * Ibb * wy;
  if constexpr (!ACC) return;
  double* tb = acc + 6 + 12;
  tb[0] += fh * Ihb + fb * Ibb;
  tb[1] += wgh * Ihb + wgb * Ibb;
  tb[2] += (H + Hp) * Ihb + (B + Bp) * Ibb;
  tb[3] += wah * H * Ihb + wab * B * Ibb;
  tb[4] += Ah * H * Ihb + Ab * B * Ibb;
  double ch = t[3] * H * Ihb, cb = t[3] * B * Ibb;
  double dh = t[4] * H * Ihb, db = t[4] * B * Ibb;
  // w bar
  acc[23] += t[1] * (Ihb * ghx + Ibb * gbx) + ch * (pax + ax[E] * kh) + cb * (pax + ax[E] * kb);
  if (D == 2) acc[24] += t[1] * (Ihb * ghy + Ibb * gby) + ch * (pay + ay[E] * kh) + cb * (pay + ay[E] * kb);
  // slope and time coefficients
  double* axb = acc + 6;
  double* ayb = acc + 10;
  double* Atb = acc + 14;
  {
    double wc = wx * (ch + cb);
    axb[0] += wc; axb[1] += wc * vx;
    if (D == 2) axb[2] += wc * vy;
    axb[E] += wx * (ch * kh + cb * kb);
    if (D == 2) {
      double wy2 = wy * (ch + cb);
      ayb[0] += wy2; ayb[1] += wy2 * vx; ayb[2] += wy2 * vy;
      ayb[E] += wy * (ch * kh + cb * kb);
    }
    double dd = dh + db;
    Atb[0] += dd; Atb[1] += dd * vx;
    if (D == 2) Atb[2] += dd * vy;
    Atb[E] += dh * kh + db * kb;
  }
  // lam through the 1/(2 lam) of the energy moments
  double il2 = -1.0 / (2.0 * e.lam * e.lam);
  double aE = wx * ax[E] + wy * ((D == 2) ? ay[E] : 0.0);
  acc[3] += (ch * 0.5 * nxi + cb * 0.5 * (nxi + 2)) * aE * il2 + (dh * 0.5 * nxi + db * 0.5 * (nxi + 2)) * At[E] * il2;
  // the equilibrium values
  double Hb = Ihb * (t[2] + t[3] * wah + t[4] * Ah), Hpb = Ihb * t[2];
  double Bb = Ibb * (t[2] + t[3] * wab + t[4] * Ab), Bpb = Ibb * t[2];
  eq_rev(g, e.rho, e.ux, e.uy, e.lam, e.qx, e.qy, vx, vy, Hb, Bb, Hpb, Bpb, acc);
}

// ------------------------------------------------------------------------
// reconstruction (Sec. 2.1, f0 = f + x . grad f, van Leer per index
// direction) and its reverse
// ------------------------------------------------------------------------
// limited index slope and its partials with respect to (low, centre, high)
// van Leer slope between two neighbouring cells and its partials
__device__ __forceinline__ double lim_vl(double vlo, double v0, double vhi, double& dlo, double& d0, double& dhi) {
  dlo = d0 = dhi = 0.0;
  const double s1 = v0 - vlo, s2 = vhi - v0;
  const double sm = s1 + s2;
  // one-sided slopes of one sign: the van Leer slope is 2 s1 s2 / (s1 + s2)
  // (|s1| + |s2| = |s1 + s2|), its partials 2 (s2 / sm)^2 and 2 (s1 / sm)^2
  // (ratios in [0, 1], so no square underflows); as in the forward pass, a
  // sum below the normal range (far tails of f) gives a zero slope
  if (s1 * s2 <= 0.0 || !(fabs(sm) >= 1e-300)) return 0.0;
  const double r = 1.0 / sm;
  const double t1 = s1 * r, t2 = s2 * r;
  const double p1 = 2.0 * t2 * t2, p2 = 2.0 * t1 * t1;
  d0 = p1 - p2; dlo = -p1; dhi = p2;
  return 2.0 * s1 * t2;
}
__device__ inline double lim_d(int lo, int hi, double vlo, double v0, double vhi, double& dlo, double& d0,
                               double& dhi) {
  dlo = d0 = dhi = 0.0;
  if (lo == kNbMiss || hi == kNbMiss) return 0.0;
  if (lo == kNbWall && hi == kNbWall) return 0.0;
  if (lo == kNbWall) { dhi = 1.0; d0 = -1.0; return vhi - v0; }
  if (hi == kNbWall) { d0 = 1.0; dlo = -1.0; return v0 - vlo; }
  return lim_vl(vlo, v0, vhi, dlo, d0, dhi);
}

__device__ __forceinline__ double nbval(const double* f, const double* finf, int code, double self, int nv, int k) {
  if (code >= 0) return f[(size_t)code * nv + k];
  if (code == kNbFar) return finf[k];
  return self;
}

// reconstructed value and physical slope of f at velocity k on the side of
// cell c whose face offset is (dx, dy); with bars (vb, gxb, gyb) the
// reverse is scattered into fb
struct SideK {
  double v, gx, gy;
};

__device__ inline SideK side_val(const Dev& g, const double* f, const double* finf, int c, double dx, double dy,
                                 int k) {
  const int* nb = g.nb + 4 * c;
  double v0 = f[(size_t)c * g.nv + k];
  double dl, d0, dh;
  double si = lim_d(nb[0], nb[1], nbval(f, finf, nb[0], v0, g.nv, k), v0, nbval(f, finf, nb[1], v0, g.nv, k), dl,
                    d0, dh);
  double sj = 0.0;
  if (kD == 2)
    sj = lim_d(nb[2], nb[3], nbval(f, finf, nb[2], v0, g.nv, k), v0, nbval(f, finf, nb[3], v0, g.nv, k), dl, d0,
               dh);
  const double* G = g.G + 4 * c;
  SideK s;
  s.gx = G[0] * si + G[1] * sj;
  s.gy = (kD == 2) ? G[2] * si + G[3] * sj : 0.0;
  s.v = v0 + s.gx * dx + s.gy * dy;
  return s;
}

__device__ __forceinline__ void scatter_code(double* fb, int code, int c, int nv, int k, double v) {
  if (code >= 0) acc_add(fb + (size_t)code * nv + k, v);
  else if (code == kNbCopy) acc_add(fb + (size_t)c * nv + k, v);
}

__device__ inline void side_rev(const Dev& g, const double* f, const double* finf, int c, double dx, double dy,
                                int k, double vb, double gxb, double gyb, double* fbar) {
  if (vb == 0.0 && gxb == 0.0 && gyb == 0.0) return;
  const int* nb = g.nb + 4 * c;
  const double* G = g.G + 4 * c;
  double v0 = f[(size_t)c * g.nv + k];
  gxb += vb * dx;
  gyb += vb * dy;
  double sib = G[0] * gxb + ((kD == 2) ? G[2] * gyb : 0.0);
  double sjb = (kD == 2) ? G[1] * gxb + G[3] * gyb : 0.0;
  double own = vb;
  for (int dir = 0; dir < kD; ++dir) {
    double sb = dir ? sjb : sib;
    int lo = nb[2 * dir], hi = nb[2 * dir + 1];
    double dl, d0, dh;
    lim_d(lo, hi, nbval(f, finf, lo, v0, g.nv, k), v0, nbval(f, finf, hi, v0, g.nv, k), dl, d0, dh);
    own += sb * d0;
    scatter_code(fbar, lo, c, g.nv, k, sb * dl);
    scatter_code(fbar, hi, c, g.nv, k, sb * dh);
  }
  acc_add(fbar + (size_t)c * g.nv + k, own);
}

// side data of face f at velocity k: cell code, centroid-to-face offset
__device__ inline void face_side(const Dev& g, const double* fp, int s, int& code, int& inner, double& dx,
                                 double& dy) {
  int L = tab_int(fp[kFpL]), R = tab_int(fp[kFpR]);
  code = s ? R : L;
  inner = (L >= 0) ? L : R;
  dx = fp[s ? kFpDR : kFpDL];
  dy = fp[(s ? kFpDR : kFpDL) + 1];
}

// value of the side distribution (ghost: far-field Maxwellian or a copy of
// the interior cell, zero slope)
__device__ inline SideK side_any(const Dev& g, const double* f, const double* finf, int code, int inner, double dx,
                                 double dy, int k) {
  if (code >= 0) return side_val(g, f, finf, code, dx, dy, k);
  SideK s;
  s.gx = s.gy = 0.0;
  s.v = (code == kNbFar) ? finf[k] : f[(size_t)inner * g.nv + k];
  return s;
}

__device__ inline void side_any_rev(const Dev& g, const double* f, const double* finf, int code, int inner,
                                    double dx, double dy, int k, double vb, double gxb, double gyb, double* fbar) {
  if (code >= 0) side_rev(g, f, finf, code, dx, dy, k, vb, gxb, gyb, fbar);
  else if (code == kNbCopy) acc_add(fbar + (size_t)inner * g.nv + k, vb);
}

// reconstruction with the partials of its two limited index slopes kept,
// for a reverse pass right after the forward evaluation
struct SideD {
  double v, gx, gy;
  double p[2][3];  // d slope / d (low, centre, high value) per index direction
};

__device__ __forceinline__ SideD side_val_d(const Dev& g, const double* f, const double* finf, int code, int inner,
                                            double dx, double dy, int k) {
  SideD s;
  for (int d = 0; d < 2; ++d) s.p[d][0] = s.p[d][1] = s.p[d][2] = 0.0;
  if (code < 0) {
    s.gx = s.gy = 0.0;
    s.v = (code == kNbFar) ? finf[k] : f[(size_t)inner * g.nv + k];
    return s;
  }
  const int* nb = g.nb + 4 * code;
  const int n0 = nb[0], n1 = nb[1], n2 = nb[2], n3 = nb[3];
  const double v0 = f[(size_t)code * g.nv + k];
  double si, sj;
  if ((n0 | n1 | n2 | n3) >= 0) {
    // four neighbouring cells (most of the field): no boundary codes to test
    const size_t nv = (size_t)g.nv;
    si = lim_vl(f[n0 * nv + k], v0, f[n1 * nv + k], s.p[0][0], s.p[0][1], s.p[0][2]);
    sj = lim_vl(f[n2 * nv + k], v0, f[n3 * nv + k], s.p[1][0], s.p[1][1], s.p[1][2]);
  } else {
    si = lim_d(n0, n1, nbval(f, finf, n0, v0, g.nv, k), v0, nbval(f, finf, n1, v0, g.nv, k), s.p[0][0], s.p[0][1],
               s.p[0][2]);
    sj = lim_d(n2, n3, nbval(f, finf, n2, v0, g.nv, k), v0, nbval(f, finf, n3, v0, g.nv, k), s.p[1][0], s.p[1][1],
               s.p[1][2]);
  }
  const double* G = g.G + 4 * code;
  s.gx = G[0] * si + G[1] * sj;
  s.gy = G[2] * si + G[3] * sj;
  s.v = v0 + s.gx * dx + s.gy * dy;
  return s;
}

__device__ __forceinline__ void side_rev_d(const Dev& g, const SideD& s, int code, int inner, double dx, double dy,
                                           int k, double vb, double gxb, double gyb, double* fbar) {
  if (code < 0) {
    if (code == kNbCopy) acc_add(fbar + (size_t)inner * g.nv + k, vb);
    return;
  }
  const int* nb = g.nb + 4 * code;
  const double* G = g.G + 4 * code;
  gxb += vb * dx;
  gyb += vb * dy;
  const double sb[2] = {G[0] * gxb + G[2] * gyb, G[1] * gxb + G[3] * gyb};
  double own = vb;
  for (int d = 0; d < 2; ++d) {
    own += sb[d] * s.p[d][1];
    const int lo = nb[2 * d], hi = nb[2 * d + 1];
    const double a = sb[d] * s.p[d][0], c = sb[d] * s.p[d][2];
    if (lo >= 0) acc_add(fbar + (size_t)lo * g.nv + k, a);
    else if (lo == kNbCopy) own += a;
    if (hi >= 0) acc_add(fbar + (size_t)hi * g.nv + k, c);
    else if (hi == kNbCopy) own += c;
  }
  acc_add(fbar + (size_t)code * g.nv + k, own);
}

// cotangent of the flux F_k (along the face normal) of face f from the
// divergence bars of its field cells and the face macro-flux bar
__device__ inline void flux_bar_k(const Dev& g, const double* fp, const double* Dbh, const double* Dbb,
                                  const double* Fbf, int k, double& Fhb, double& Fbb) {
  int L = tab_int(fp[kFpL]), R = tab_int(fp[kFpR]);
  double S = fp[kFpS];
  double vx = g.vx[k], vy = g.vy[k], w = g.wk[k];
  Fhb = w * (Fbf[0] + Fbf[1] * vx + ((kD == 2) ? Fbf[2] * vy : 0.0) + Fbf[kD + 1] * 0.5 * (vx * vx + vy * vy));
  Fbb = w * 0.5 * Fbf[kD + 1];
  if (L >= 0 && g.type[L] == 1) {
    double a = -S / g.vol[L];
    Fhb += a * Dbh[(size_t)L * g.nv + k];
    Fbb += a * Dbb[(size_t)L * g.nv + k];
  }
  if (R >= 0 && g.type[R] == 1) {
    double a = S / g.vol[R];
    Fhb += a * Dbh[(size_t)R * g.nv + k];
    Fbb += a * Dbb[(size_t)R * g.nv + k];
  }
}

// ------------------------------------------------------------------------
// the face reverses run one face per block of up to kFaceWaves wavefronts,
// threads over velocities
// ------------------------------------------------------------------------
constexpr int kFaceWaves = 8;

// sum over the block of each thread's v[0..N-1], returned to every thread:
// the wavefront sums, then those in wavefront order (a fixed order).  Every
// thread of the block must call it; red holds kFaceWaves * N doubles.
template <int N>
__device__ __forceinline__ void block_sum(double* v, double* red) {
  for (int i = 0; i < N; ++i) v[i] = wave_sum(v[i]);
  const int nwv = blockDim.x >> 6;
  if (nwv == 1) return;
  const int wv = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0)
    for (int i = 0; i < N; ++i) red[wv * N + i] = v[i];
  __syncthreads();
  for (int i = 0; i < N; ++i) {
    double t = red[i];
    for (int w = 1; w < nwv; ++w) t += red[w * N + i];
    v[i] = t;
  }
}

// ------------------------------------------------------------------------
// flux reverse, faces between cells (interior and ghost faces): one block
// per face, threads over velocities.  The face record lives in LDS (the
// first wavefront computes it from the block sums).  Pass 1: W0; pass 2:
// q0 and the sums of its U-derivative; pass 3: the flux reversed per
// velocity (its bars of the upwind data scattered at once) with the record
// bars accumulated; the record Jacobian in the first wavefront, one input
// per lane;
// pass 4: the moment bars (W0, q0) scattered to both sides.
// ------------------------------------------------------------------------
__device__ __forceinline__ void store_rec(Rec& e, double rho, double ux, double uy, double lam, double qx, double qy,
                                          const double* c) {
  e.rho = rho; e.ux = ux; e.uy = uy; e.lam = lam; e.qx = qx; e.qy = qy;
  for (int i = 0; i < kRecOut; ++i) e.c[i] = c[i];
}

__device__ __forceinline__ void rec_values(const Dev& g, double dts, const double* x, double* c) {
  face_coeffs(g, dts, x, c);
}

// sc: this workgroup's [6][nv] staging of the pass-3 bars of the upwind
// reconstructions (value, physical slopes; h then b), completed by the
// moment bars in pass 4 and scattered once
__device__ __forceinline__ void adj_face_body(const Dev& g, int f, double dts, const double* __restrict__ h,
                                              const double* __restrict__ b, const double* __restrict__ gW,
                                              const double* __restrict__ rec, const double* __restrict__ Dbh,
                                              const double* __restrict__ Dbb, const double* __restrict__ Fb,
                                              double* __restrict__ hbar, double* __restrict__ bbar,
                                              double* __restrict__ gWbar, double* __restrict__ fbar,
                                              double* __restrict__ sc, Rec& e, double* sred, double* sxb) {
  const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63;
  const double* fp = g.fplan + (size_t)f * kFpN;
  if (tab_int(fp[kFpAct]) == 0) return;
  const int L = tab_int(fp[kFpL]), R = tab_int(fp[kFpR]);
  if (L == kNbWall || R == kNbWall) return;
  const int D = kD, nv = g.nv;
  const double nx = fp[kFpN0], ny = fp[kFpN0 + 1], ufx = fp[kFpU], ufy = fp[kFpU + 1];
  const double* hinf = (const double*)g.finf_h;
  const double* binf = (const double*)g.finf_b;
  int cL, cR, inner;
  double dLx, dLy, dRx, dRy;
  face_side(g, fp, 0, cL, inner, dLx, dLy);
  face_side(g, fp, 1, cR, inner, dRx, dRy);
  // upwind interface data (the mean of both sides on a tie); the side is
  // chosen per lane, so the wavefront runs one reconstruction per component
  auto upwind = [&](int k, double wn, double& fh, double& fb) {
    const bool lft = wn > 0.0;
    const int up = lft ? cL : cR;
    const double ox = lft ? dLx : dRx, oy = lft ? dLy : dRy;
    fh = side_any(g, h, hinf, up, inner, ox, oy, k).v;
    fb = side_any(g, b, binf, up, inner, ox, oy, k).v;
    if (wn == 0.0) {
      fh = 0.5 * (fh + side_any(g, h, hinf, cL, inner, dLx, dLy, k).v);
      fb = 0.5 * (fb + side_any(g, b, binf, cL, inner, dLx, dLy, k).v);
    }
  };
  auto grad_in = [&](double* x) {
    for (int m = 0; m < 8; ++m) {
      double gl = (L >= 0) ? gW[(size_t)L * 8 + m] : 0.0;
      double gr = (R >= 0) ? gW[(size_t)R * 8 + m] : 0.0;
      x[4 + m] = 0.5 * (gl + gr);
    }
    x[12] = ufx; x[13] = ufy;
  };
  double W0[4] = {0, 0, 0, 0};
  double T1, Txx, Tyy, Txy;
  {
    // pass 1: velocity moments of the upwind interface data about the shift
    // sx, sy (the mean velocity of the face's two sides), up to third order
    // for h and first order for b; W0, q0 and the U-derivative sums of q0
    // follow from them
    const double* fr = rec + (size_t)f * NREC;
    const double sx = fr[R_SX], sy = fr[R_SY];
    double m[13];
    for (int i = 0; i < 13; ++i) m[i] = 0.0;
    for (int k = tid; k < nv; k += nt) {
      double vx = g.vx[k], vy = g.vy[k], w = g.wk[k];
      double fh, fb;
      upwind(k, wn_exact(vx, vy, ufx, ufy, nx, ny), fh, fb);
      const double cx = vx - sx, cy = vy - sy;
      const double a0 = w * fh, ax = a0 * cx, ay = a0 * cy;
      m[0] += a0; m[1] += ax; m[2] += ay;
      m[3] += ax * cx; m[4] += ax * cy; m[5] += ay * cy;
      m[6] += ax * cx * cx; m[7] += ax * cx * cy; m[8] += ax * cy * cy; m[9] += ay * cy * cy;
      const double b0 = w * fb;
      m[10] += b0; m[11] += b0 * cx; m[12] += b0 * cy;
    }
    block_sum<13>(m, sred);
    const double M0 = m[0], M1x = m[1], M1y = m[2], Mxx = m[3], Mxy = m[4], Myy = m[5];
    const double Mxxx = m[6], Mxxy = m[7], Mxyy = m[8], Myyy = m[9], B0 = m[10], B1x = m[11], B1y = m[12];
    W0[0] = M0;
    W0[1] = M1x + sx * M0;
    W0[2] = M1y + sy * M0;
    W0[3] = 0.5 * (Mxx + Myy + 2.0 * (sx * M1x + sy * M1y) + (sx * sx + sy * sy) * M0) + 0.5 * B0;
    double rho, ux, uy, lam;
    prim_d(D, kNxi, W0, rho, ux, uy, lam);
    // c = v - U0 = (v - s) - d with d = U0 - s
    const double dx = ux - sx, dy = uy - sy, d2 = dx * dx + dy * dy;
    const double dM1 = dx * M1x + dy * M1y;
    const double q0x = 0.5 * ((Mxxx + Mxyy) - 2.0 * (dx * Mxx + dy * Mxy) + d2 * M1x - dx * (Mxx + Myy) +
                              2.0 * dx * dM1 - dx * d2 * M0 + B1x - dx * B0);
    const double q0y = 0.5 * ((Mxxy + Myyy) - 2.0 * (dx * Mxy + dy * Myy) + d2 * M1y - dy * (Mxx + Myy) +
                              2.0 * dy * dM1 - dy * d2 * M0 + B1y - dy * B0);
    T1 = (Mxx + Myy) - 2.0 * dM1 + d2 * M0 + B0;
    Txx = Mxx - 2.0 * dx * M1x + dx * dx * M0;
    Tyy = Myy - 2.0 * dy * M1y + dy * dy * M0;
    Txy = Mxy - dx * M1y - dy * M1x + dx * dy * M0;
    double x[kRecIn], c[kRecOut];
    x[0] = rho; x[1] = ux; x[2] = uy; x[3] = lam;
    grad_in(x);
    if (tid < 64) {
      rec_values(g, dts, x, c);
      store_rec(e, rho, ux, uy, lam, q0x, q0y, c);
    }
    __syncthreads();
  }
  // pass 3: reverse of the flux at every velocity; the bars of the upwind
  // data go to the cells at once, the record bars are accumulated
  double acc[kRecBar];
  for (int i = 0; i < kRecBar; ++i) acc[i] = 0.0;
  double ufb_x = 0.0, ufb_y = 0.0;
  const double* Fbf = Fb + (size_t)f * kNw;
  for (int k = tid; k < nv; k += nt) {
    double vx = g.vx[k], vy = g.vy[k];
    double wn = wn_exact(vx, vy, ufx, ufy, nx, ny);
    if (wn == 0.0) continue;
    double Fhb, Fbb;
    flux_bar_k(g, fp, Dbh, Dbb, Fbf, k, Fhb, Fbb);
    const bool lft = wn > 0.0;
    const int up = lft ? cL : cR;
    const double ox = lft ? dLx : dRx, oy = lft ? dLy : dRy;
    SideD sh = side_val_d(g, h, hinf, up, inner, ox, oy, k), sb = side_val_d(g, b, binf, up, inner, ox, oy, k);
    double fhb, fbb, ghb[2], gbb[2], Ih, Ib;
    iint_rev<true>(g, e, vx, vy, vx - ufx, (D == 2) ? vy - ufy : 0.0, sh.v, sb.v, sh.gx, sh.gy, sb.gx, sb.gy,
                   Fhb * wn / dts, Fbb * wn / dts, fhb, fbb, ghb, gbb, acc, Ih, Ib);
    double wnb = (Fhb * Ih + Fbb * Ib) / dts;
    ufb_x -= wnb * nx;
    ufb_y -= wnb * ny;
    sc[k] = fhb; sc[nv + k] = ghb[0]; sc[2 * nv + k] = ghb[1];
    sc[3 * nv + k] = fbb; sc[4 * nv + k] = gbb[0]; sc[5 * nv + k] = gbb[1];
  }
  block_sum<kRecBar>(acc, sred);
  {
    double v[2] = {ufb_x, ufb_y};
    block_sum<2>(v, sred);
    ufb_x = v[0] - acc[23];
    ufb_y = v[1] - acc[24];
  }
  // contraction with the record Jacobian: lane j < kRecIn holds input j's bar
  double xb[kRecIn];
  if (tid < 64) {
    double x[kRecIn], val[kRecOut], col[kRecOut];
    x[0] = e.rho; x[1] = e.ux; x[2] = e.uy; x[3] = e.lam;
    grad_in(x);
    face_coeffs_lanes(g, dts, x, lane, val, col);
    double inb = 0.0;
    for (int i = 0; i < kRecOut; ++i) inb += acc[6 + i] * col[i];
    if (lane < kRecIn) sxb[lane] = inb;
  }
  __syncthreads();
  for (int j = 0; j < kRecIn; ++j) xb[j] = sxb[j];
  double uxb = acc[1] + xb[1], uyb = acc[2] + xb[2];
  const double qxb = acc[4], qyb = acc[5];
  ufb_x += xb[12];
  ufb_y += xb[13];
  // q0 depends on U0 through c = v - U0
  uxb += -0.5 * (T1 + 2.0 * Txx) * qxb - Txy * qyb;
  if (D == 2) uyb += -Txy * qxb - 0.5 * (T1 + 2.0 * Tyy) * qyb;
  double W0b[4] = {0, 0, 0, 0};
  prim_rev(D, kNxi, W0, acc[0] + xb[0], uxb, uyb, acc[3] + xb[3], W0b);
  // gradient bars of the two cells (the face slope is their mean)
  if (tid < 8) {
    double v = 0.5 * xb[4 + lane];
    if (L >= 0) acc_add(gWbar + (size_t)L * 8 + lane, v);
    if (R >= 0) acc_add(gWbar + (size_t)R * 8 + lane, v);
  }
  if (tid == 0) {
    fbar[(size_t)f * 5 + 0] += ufb_x;
    fbar[(size_t)f * 5 + 1] += ufb_y;
  }
  // pass 4: the moment bars of the upwind data (W0, q0) added to the staged
  // pass-3 bars, one scatter of the upwind reconstruction per velocity (on a
  // tie, which pass 3 skips: half to each side)
  const double ux0 = e.ux, uy0 = e.uy;
  for (int k = tid; k < nv; k += nt) {
    double vx = g.vx[k], vy = g.vy[k], w = g.wk[k];
    double wn = wn_exact(vx, vy, ufx, ufy, nx, ny);
    double cx = vx - ux0, cy = (D == 2) ? vy - uy0 : 0.0;
    double cqb = cx * qxb + cy * qyb;
    double mh = w * (W0b[0] + W0b[1] * vx + ((D == 2) ? W0b[2] * vy : 0.0) +
                     W0b[D + 1] * 0.5 * (vx * vx + vy * vy)) + w * 0.5 * cqb * (cx * cx + cy * cy);
    double mb = w * 0.5 * W0b[D + 1] + w * 0.5 * cqb;
    // the upwind side, chosen per lane
    const bool lft = wn > 0.0;
    const int up = lft ? cL : cR;
    const double ox = lft ? dLx : dRx, oy = lft ? dLy : dRy;
    if (wn == 0.0) {
      side_any_rev(g, h, hinf, up, inner, ox, oy, k, 0.5 * mh, 0.0, 0.0, hbar);
      side_any_rev(g, b, binf, up, inner, ox, oy, k, 0.5 * mb, 0.0, 0.0, bbar);
      side_any_rev(g, h, hinf, cL, inner, dLx, dLy, k, 0.5 * mh, 0.0, 0.0, hbar);
      side_any_rev(g, b, binf, cL, inner, dLx, dLy, k, 0.5 * mb, 0.0, 0.0, bbar);
    } else {
      const SideD sh = side_val_d(g, h, hinf, up, inner, ox, oy, k);
      side_rev_d(g, sh, up, inner, ox, oy, k, sc[k] + mh, sc[nv + k], sc[2 * nv + k], hbar);
      const SideD sb = side_val_d(g, b, binf, up, inner, ox, oy, k);
      side_rev_d(g, sb, up, inner, ox, oy, k, sc[3 * nv + k] + mb, sc[4 * nv + k], sc[5 * nv + k], bbar);
    }
  }
}

// one face per workgroup (sc: kFaceBlocks x [6][nv]; at most kFaceBlocks
// workgroups per launch)
__global__ __launch_bounds__(64 * kFaceWaves) void k_adj_face(Dev g, const int* __restrict__ items, int nitems,
                                                              double dts, const double* __restrict__ h,
                                                              const double* __restrict__ b,
                                                              const double* __restrict__ gW,
                                                              const double* __restrict__ rec,
                                                              const double* __restrict__ Dbh,
                                                              const double* __restrict__ Dbb,
                                                              const double* __restrict__ Fb, double* __restrict__ hbar,
                                                              double* __restrict__ bbar, double* __restrict__ gWbar,
                                                              double* __restrict__ fbar, double* __restrict__ fsc) {
  __shared__ Rec e;
  __shared__ double sred[kFaceWaves * kRecBar];
  __shared__ double sxb[kRecIn];
  if ((int)blockIdx.x >= nitems) return;
  adj_face_body(g, items[blockIdx.x], dts, h, b, gW, rec, Dbh, Dbb, Fb, hbar, bbar, gWbar, fbar,
                fsc + (size_t)blockIdx.x * 6 * g.nv, e, sred, sxb);
}

// ------------------------------------------------------------------------
// flux reverse, isothermal wall faces (Eq. maxWalldes): one wavefront per
// face.  Pass 1: incident mass flux and the wall normaliser; pass 2: the
// reflected part reversed (bars of rho_w, T_w, v_w, U_f); pass 3: the
// incident part reversed, its bars scattered at once, record bars
// accumulated; then the record Jacobian and the incident state.
// ------------------------------------------------------------------------
__global__ __launch_bounds__(64 * kFaceWaves) void k_adj_wall(Dev g, const int* __restrict__ items, int nitems, double dts,
                                                  const double* __restrict__ h,
                                                  const double* __restrict__ b, const double* __restrict__ W,
                                                  const double* __restrict__ q, const double* __restrict__ gW,
                                                  const double* __restrict__ Dbh, const double* __restrict__ Dbb,
                                                  const double* __restrict__ Fb, double* __restrict__ hbar,
                                                  double* __restrict__ bbar, double* __restrict__ Wbar,
                                                  double* __restrict__ qbar, double* __restrict__ gWbar,
                                                  double* __restrict__ fbar) {
  __shared__ Rec e;
  __shared__ double sred[kFaceWaves * kRecBar];
  __shared__ double sxb[kRecIn];
  const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63;
  if ((int)blockIdx.x >= nitems) return;
  const int f = items[blockIdx.x];
  const int L = g.fcell[2 * f], R = g.fcell[2 * f + 1];
  if (L != kNbWall && R != kNbWall) return;
  const int c = (L == kNbWall) ? R : L;
  if (c < 0 || g.type[c] != 1) return;
  const int D = kD, nw = kNw, nv = g.nv, nxi = kNxi;
  int fs = 0;
  for (int s = 0; s < 4; ++s) if (g.cf[4 * c + s] == f) fs = s;
  const double* fg = g.fgeo + (size_t)f * 8;
  const double sgn = (R == kNbWall) ? 1.0 : -1.0;
  const double nwx = sgn * fg[0], nwy = sgn * fg[1], ufx = fg[3], ufy = fg[4];
  const double vwx = fg[5], vwy = fg[6], rtw = fg[7];
  const double dx = g.cdx[8 * c + 2 * fs], dy = g.cdx[8 * c + 2 * fs + 1];
  const double* hinf = (const double*)g.finf_h;
  const double* binf = (const double*)g.finf_b;
  // incident state: one-sided extrapolation of W, cell state if unphysical
  const double* gw = gW + (size_t)c * 8;
  double Win[4] = {0, 0, 0, 0};
  for (int m = 0; m < nw; ++m) Win[m] = W[(size_t)c * nw + m] + gw[m] * dx + gw[nw + m] * dy;
  const bool extrap = physical_state(D, Win);
  if (!extrap)
    for (int m = 0; m < nw; ++m) Win[m] = W[(size_t)c * nw + m];
  auto rec_in = [&](double* x) {
    prim_d(D, nxi, Win, x[0], x[1], x[2], x[3]);
    for (int m = 0; m < 8; ++m) x[4 + m] = gw[m];
    x[12] = ufx; x[13] = ufy;
  };
  {
    double x[kRecIn], cc[kRecOut];
    rec_in(x);
    if (tid < 64) {
      rec_values(g, dts, x, cc);
      store_rec(e, x[0], x[1], x[2], x[3], q[(size_t)c * D], (D == 2) ? q[(size_t)c * D + 1] : 0.0, cc);
    }
    __syncthreads();
  }
  const double lamw = 0.5 / rtw;
  const double nrm = pow(lamw / kPi, 0.5 * D);
  const double betaw = (double)nxi / (2.0 * lamw);
  // pass 1: incident mass flux and the wall normaliser
  double num = 0.0, den = 0.0;
  for (int k = tid; k < nv; k += nt) {
    double vx = g.vx[k], vy = g.vy[k], w = g.wk[k];
    double wn = wn_exact(vx, vy, ufx, ufy, nwx, nwy);
    if (wn > 0.0) {
      SideK sh = side_val(g, h, hinf, c, dx, dy, k), sb = side_val(g, b, binf, c, dx, dy, k);
      double fhb, fbb, ghb[2], gbb[2], Ih, Ib;
      iint_rev<false>(g, e, vx, vy, vx - ufx, (D == 2) ? vy - ufy : 0.0, sh.v, sb.v, sh.gx, sh.gy, sb.gx, sb.gy,
                      0.0, 0.0, fhb, fbb, ghb, gbb, nullptr, Ih, Ib);
      num += w * wn * Ih;
    } else if (wn < 0.0) {
      double cx = vx - vwx, cy = (D == 2) ? vy - vwy : 0.0;
      den += w * wn * nrm * exp(-lamw * (cx * cx + cy * cy));
    }
  }
  {
    double v[2] = {num, den};
    block_sum<2>(v, sred);
    num = v[0];
    den = v[1];
  }
  const double rhow = -num / (dts * den);
  const double* Fbf = Fb + (size_t)f * nw;
  const double* fpw = g.fplan + (size_t)f * kFpN;
  // pass 2: the reflected part (wn < 0) and the normaliser's derivatives
  double rhowb = 0, lamwb = 0, vwbx = 0, vwby = 0, ufbx = 0, ufby = 0;
  double dden_l = 0, dden_vx = 0, dden_vy = 0, dden_u = 0;
  for (int k = tid; k < nv; k += nt) {
    double vx = g.vx[k], vy = g.vy[k], w = g.wk[k];
    double wn = wn_exact(vx, vy, ufx, ufy, nwx, nwy);
    if (!(wn < 0.0)) continue;
    double Fhb, Fbb;
    flux_bar_k(g, fpw, Dbh, Dbb, Fbf, k, Fhb, Fbb);
    double fhb = sgn * Fhb, fbb = sgn * Fbb;
    double cx = vx - vwx, cy = (D == 2) ? vy - vwy : 0.0;
    double c2 = cx * cx + cy * cy;
    double Ek = nrm * exp(-lamw * c2);
    double Hw = rhow * Ek;
    double t = fhb + fbb * betaw;
    rhowb += t * wn * Ek;
    lamwb += fhb * wn * Hw * (0.5 * D / lamw - c2) + fbb * wn * betaw * Hw * (0.5 * D / lamw - c2 - 1.0 / lamw);
    vwbx += t * wn * Hw * 2.0 * lamw * cx;
    vwby += t * wn * Hw * 2.0 * lamw * cy;
    ufbx -= t * Hw * nwx;
    ufby -= t * Hw * nwy;
    dden_l += w * wn * Ek * (0.5 * D / lamw - c2);
    dden_vx += w * wn * Ek * 2.0 * lamw * cx;
    dden_vy += w * wn * Ek * 2.0 * lamw * cy;
    dden_u += w * Ek;
  }
  {
    double v[10] = {rhowb, lamwb, vwbx, vwby, ufbx, ufby, dden_l, dden_vx, dden_vy, dden_u};
    block_sum<10>(v, sred);
    rhowb = v[0]; lamwb = v[1];
    vwbx = v[2]; vwby = v[3];
    ufbx = v[4]; ufby = v[5];
    dden_l = v[6]; dden_vx = v[7]; dden_vy = v[8]; dden_u = v[9];
  }
  const double numb = -rhowb / (dts * den);
  const double denb = -rhowb * rhow / den;
  lamwb += denb * dden_l;
  vwbx += denb * dden_vx;
  vwby += denb * dden_vy;
  ufbx -= denb * dden_u * nwx;
  ufby -= denb * dden_u * nwy;
  // pass 3: incident part (wn > 0): bars of the incident data scattered,
  // record bars accumulated
  double acc[kRecBar];
  for (int i = 0; i < kRecBar; ++i) acc[i] = 0.0;
  double ufb2x = 0, ufb2y = 0;
  for (int k = tid; k < nv; k += nt) {
    double vx = g.vx[k], vy = g.vy[k], w = g.wk[k];
    double wn = wn_exact(vx, vy, ufx, ufy, nwx, nwy);
    if (!(wn > 0.0)) continue;
    double Fhb, Fbb;
    flux_bar_k(g, fpw, Dbh, Dbb, Fbf, k, Fhb, Fbb);
    double fhb_ = sgn * Fhb, fbb_ = sgn * Fbb;
    SideD sh = side_val_d(g, h, hinf, c, c, dx, dy, k), sb = side_val_d(g, b, binf, c, c, dx, dy, k);
    double Ihb = fhb_ * wn / dts + numb * w * wn, Ibb = fbb_ * wn / dts;
    double fhb, fbb, ghb[2], gbb[2], Ih, Ib;
    iint_rev<true>(g, e, vx, vy, vx - ufx, (D == 2) ? vy - ufy : 0.0, sh.v, sb.v, sh.gx, sh.gy, sb.gx, sb.gy, Ihb,
                   Ibb, fhb, fbb, ghb, gbb, acc, Ih, Ib);
    double wnb = fhb_ * Ih / dts + fbb_ * Ib / dts + numb * w * Ih;
    ufb2x -= wnb * nwx;
    ufb2y -= wnb * nwy;
    side_rev_d(g, sh, c, c, dx, dy, k, fhb, ghb[0], ghb[1], hbar);
    side_rev_d(g, sb, c, c, dx, dy, k, fbb, gbb[0], gbb[1], bbar);
  }
  block_sum<kRecBar>(acc, sred);
  {
    double v[2] = {ufb2x, ufb2y};
    block_sum<2>(v, sred);
    ufbx += v[0] - acc[23];
    ufby += v[1] - acc[24];
  }
  double xb[kRecIn];
  if (tid < 64) {
    double x[kRecIn], val[kRecOut], col[kRecOut];
    rec_in(x);
    face_coeffs_lanes(g, dts, x, lane, val, col);
    double inb = 0.0;
    for (int i = 0; i < kRecOut; ++i) inb += acc[6 + i] * col[i];
    if (lane < kRecIn) sxb[lane] = inb;
  }
  __syncthreads();
  for (int j = 0; j < kRecIn; ++j) xb[j] = sxb[j];
  ufbx += xb[12];
  ufby += xb[13];
  double Winb[4] = {0, 0, 0, 0};
  prim_rev(D, nxi, Win, acc[0] + xb[0], acc[1] + xb[1], acc[2] + xb[2], acc[3] + xb[3], Winb);
  if (tid == 0) {
    acc_add(qbar + (size_t)c * D, acc[4]);
    if (D == 2) acc_add(qbar + (size_t)c * D + 1, acc[5]);
    for (int m = 0; m < nw; ++m) acc_add(Wbar + (size_t)c * nw + m, Winb[m]);
    double* o = fbar + (size_t)f * 5;
    o[0] += ufbx; o[1] += ufby;
    o[2] += vwbx; o[3] += vwby;
    o[4] += -lamwb * 2.0 * lamw * lamw;  // lam_w = 1/(2 RT_w)
  }
  if (tid < 8) {
    // the slope input and, through the extrapolation, the incident state
    double v = xb[4 + lane];
    if (extrap) {
      if (lane < nw) v += Winb[lane] * dx;
      else if (lane >= nw && lane < 2 * nw) v += Winb[lane - nw] * dy;
    }
    acc_add(gWbar + (size_t)c * 8 + lane, v);
  }
}

// ------------------------------------------------------------------------
// limited W gradients (reconstruction of W for the slopes and the wall
// incident state): gW bars to W bars, one thread per cell
// ------------------------------------------------------------------------
__global__ void k_adj_gradW(Dev g, const int* __restrict__ items, int nitems, const double* __restrict__ W,
                            const double* __restrict__ gWbar, double* __restrict__ Wbar) {
  const int slot = blockIdx.x * blockDim.x + threadIdx.x;
  if (slot >= nitems) return;
  const int c = items[slot];
  if (g.type[c] == 0) return;
  const int nw = kNw;
  const double* gb = gWbar + (size_t)c * 8;
  const double* G = g.G + 4 * c;
  const int* nb = g.nb + 4 * c;
  for (int m = 0; m < nw; ++m) {
    double gxb = gb[m], gyb = (kD == 2) ? gb[nw + m] : 0.0;
    double sib = G[0] * gxb + ((kD == 2) ? G[2] * gyb : 0.0);
    double sjb = (kD == 2) ? G[1] * gxb + G[3] * gyb : 0.0;
    double v0 = W[(size_t)c * nw + m];
    auto val = [&](int code) -> double {
      if (code >= 0) return W[(size_t)code * nw + m];
      if (code == kNbFar) return g.winf[m];
      return v0;
    };
    double own = 0.0;
    for (int dir = 0; dir < kD; ++dir) {
      double sb = dir ? sjb : sib;
      if (sb == 0.0) continue;
      int lo = nb[2 * dir], hi = nb[2 * dir + 1];
      double dl, d0, dh;
      lim_d(lo, hi, val(lo), v0, val(hi), dl, d0, dh);
      own += sb * d0;
      if (lo >= 0) acc_add(Wbar + (size_t)lo * nw + m, sb * dl);
      else if (lo == kNbCopy) own += sb * dl;
      if (hi >= 0) acc_add(Wbar + (size_t)hi * nw + m, sb * dh);
      else if (hi == kNbCopy) own += sb * dh;
    }
    acc_add(Wbar + (size_t)c * nw + m, own);
  }
}

// ------------------------------------------------------------------------
// Step 7 (W' = W~ + sum_k V_k Psi_k (f' - g(W~))) and the heat flux of the
// new state, reversed: one wavefront per cell.  hb, bb hold the bars of f'
// on entry and on return (plus the contributions of these two maps); Wpb
// receives the bar of the macro predictor W~.
// ------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_adj_step7(Dev g, const double* __restrict__ h1,
                                                   const double* __restrict__ b1, const double* __restrict__ W1,
                                                   const double* __restrict__ Wp, const double* __restrict__ W1b,
                                                   const double* __restrict__ q1b, double* __restrict__ hb,
                                                   double* __restrict__ bb, double* __restrict__ Wpb) {
  const int c = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (c >= g.ncell) return;
  const int D = kD, nw = kNw, nv = g.nv;
  double Wb[4] = {0, 0, 0, 0};
  for (int m = 0; m < nw; ++m) Wb[m] = W1b[(size_t)c * nw + m];
  if (g.type[c] == 0) {
    if (lane < nw) Wpb[(size_t)c * nw + lane] = Wb[lane];
    return;
  }
  // q' = heat flux of f' about the velocity of W'
  double rho1, ux1, uy1, lam1;
  prim_d(D, kNxi, W1 + (size_t)c * nw, rho1, ux1, uy1, lam1);
  const double qxb = q1b[(size_t)c * D], qyb = (D == 2) ? q1b[(size_t)c * D + 1] : 0.0;
  double uxb = 0.0, uyb = 0.0;
  for (int k = lane; k < nv; k += 64) {
    size_t o = (size_t)c * nv + k;
    double dh, db;
    heat_rev_k(D, g.wk[k], g.vx[k], g.vy[k], ux1, uy1, h1[o], b1[o], qxb, qyb, dh, db, uxb, uyb);
    hb[o] += dh;
    bb[o] += db;
  }
  uxb = wave_sum(uxb);
  uyb = wave_sum(uyb);
  prim_rev(D, kNxi, W1 + (size_t)c * nw, 0.0, uxb, uyb, 0.0, Wb);
  if (g.type[c] != 1) {
    if (lane < nw) Wpb[(size_t)c * nw + lane] = Wb[lane];
    return;
  }
  double rho, ux, uy, lam;
  prim_d(D, kNxi, Wp + (size_t)c * nw, rho, ux, uy, lam);
  double a[6] = {0, 0, 0, 0, 0, 0};
  for (int k = lane; k < nv; k += 64) {
    size_t o = (size_t)c * nv + k;
    double vx = g.vx[k], vy = g.vy[k], w = g.wk[k];
    double P = Wb[0] + Wb[1] * vx + ((D == 2) ? Wb[2] * vy : 0.0) + Wb[D + 1] * 0.5 * (vx * vx + vy * vy);
    double Pb = 0.5 * Wb[D + 1];
    hb[o] += w * P;
    bb[o] += w * Pb;
    eq_rev(g, rho, ux, uy, lam, 0.0, 0.0, vx, vy, -w * P, -w * Pb, 0.0, 0.0, a);
  }
  for (int i = 0; i < 4; ++i) a[i] = wave_sum(a[i]);
  double Wpbl[4] = {Wb[0], Wb[1], Wb[2], Wb[3]};
  prim_rev(D, kNxi, Wp + (size_t)c * nw, a[0], a[1], a[2], a[3], Wpbl);
  if (lane < nw) Wpb[(size_t)c * nw + lane] = Wpbl[lane];
}

// ------------------------------------------------------------------------
// micro LU-SGS reversed (Eq. dualTimeStepping_micro).  With the forward
// sweeps x = (D+U)^{-1} D (D+L)^{-1} r, the bar of the residual is
// r_bar = (D+L)^{-T} D (D+U)^{-T} x_bar: an ascending transposed sweep for
// y = (D+U)^{-T} x_bar, then a descending one for r_bar.  One workgroup per
// block and 16-velocity chunk, groups of 16 lanes over the rows of a
// hyperplane.
// ------------------------------------------------------------------------
__device__ __forceinline__ double micro_coef(const double* mg, int s, double vx, double vy) {
  return mg[3 * s] * vx + mg[3 * s + 1] * vy - mg[3 * s + 2];
}

template <int MODE>
__global__ __launch_bounds__(1024) void k_adj_micro_sweep(Dev g, const int* __restrict__ binfo,
                                                          const double* __restrict__ crec,
                                                          const double* __restrict__ inh,
                                                          const double* __restrict__ inb,
                                                          double* __restrict__ outh, double* __restrict__ outb) {
  // 16 velocities per workgroup (one per lane of a 16-lane group), the
  // groups over the rows of a hyperplane
  const int blk = blockIdx.x;
  const int wave = threadIdx.x >> 4, nwav = blockDim.x >> 4;
  const int k = blockIdx.y * 16 + (threadIdx.x & 15);
  const int ni = binfo[8 * blk], nj = binfo[8 * blk + 1], c0 = binfo[8 * blk + 2];
  const bool kok = k < g.nv;
  const int kk = kok ? k : 0;
  const double vx = g.vx[kk], vy = g.vy[kk];
  const int nh = ni + nj - 1;
  const int ns = 2 * kD;
  for (int it = 0; it < nh; ++it) {
    const int hp = (MODE == 0) ? it : nh - 1 - it;
    for (int j = wave; j < nj; j += nwav) {
      const int i = hp - j;
      if (i < 0 || i >= ni || !kok) continue;
      const int n = c0 + i + ni * j;
      if (g.type[n] != 1) continue;
      const double* mg = g.mgeo + (size_t)n * 12;
      double dd = crec[(size_t)n * NCREC + C_D0];
      for (int s = 0; s < ns; ++s) dd += fmax(micro_coef(mg, s, vx, vy), 0.0);
      double sh = 0.0, sb = 0.0;
      for (int s = 0; s < ns; ++s) {
        const int m = g.nb[4 * n + s];
        if (m < 0 || g.type[m] != 1) continue;
        if ((MODE == 0) ? (m < n) : (m > n)) {
          const double cf = fmin(micro_coef(g.mgeo + (size_t)m * 12, s ^ 1, vx, vy), 0.0);
          sh += cf * outh[(size_t)m * g.nv + k];
          sb += cf * outb[(size_t)m * g.nv + k];
        }
      }
      const size_t o = (size_t)n * g.nv + k;
      if (MODE == 0) {
        outh[o] = (inh[o] - sh) / dd;
        outb[o] = (inb[o] - sb) / dd;
      } else {
        outh[o] = inh[o] - sh / dd;
        outb[o] = inb[o] - sb / dd;
      }
    }
    __syncthreads();
  }
}

// Coefficient and residual bars of the micro step, one wavefront per cell:
// with x = f' - f (the micro increment), x* the forward-sweep result, y and
// r_bar from the two transposed sweeps, the bars of the diagonal d, of the
// lower couplings L (cell n, neighbour m < n) and the upper couplings U are
//   d_bar = -r_bar x + (y - r_bar)(x* - x),  L_bar = -r_bar_n x*_m,
//   U_bar = -y_n x_m,
// summed over h and b.  Then the residual r = S - f/dt + (D + (f+ - f)/tau)/2
// is reversed (its f+ through the Shakhov equilibrium of (W~, q~)), and q~,
// the heat flux of f about the velocity of W~.
__global__ __launch_bounds__(256, 2) void k_adj_micro_coef(
    Dev g, double dt, const double* __restrict__ crec, const double* __restrict__ Wp,
    const double* __restrict__ h0, const double* __restrict__ b0, const double* __restrict__ h1,
    const double* __restrict__ b1, const double* __restrict__ xsh, const double* __restrict__ xsb,
    const double* __restrict__ yh, const double* __restrict__ yb, const double* __restrict__ rh,
    const double* __restrict__ rb, const double* __restrict__ xbh, const double* __restrict__ xbb,
    double* __restrict__ hbar, double* __restrict__ bbar, double* __restrict__ Shb, double* __restrict__ Sbb,
    double* __restrict__ Dbh, double* __restrict__ Dbb, double* __restrict__ Wpb, double* __restrict__ sbar) {
  const int c = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (c >= g.ncell) return;
  const int D = kD, nv = g.nv, nw = kNw, ns = 2 * D;
  if (g.type[c] != 1) {
    for (int k = lane; k < nv; k += 64) {
      size_t o = (size_t)c * nv + k;
      hbar[o] = xbh[o];
      bbar[o] = xbb[o];
      Shb[o] = 0.0; Sbb[o] = 0.0; Dbh[o] = 0.0; Dbb[o] = 0.0;
    }
    return;
  }
  const double* r = crec + (size_t)c * NCREC;
  const double rho = r[C_RHO], ux = r[C_UX], uy = r[C_UY], lam = r[C_LAM], qx = r[C_QX], qy = r[C_QY];
  const double it = r[C_ITAU];
  const double* mg = g.mgeo + (size_t)c * 12;
  int nbm[4];
  for (int s = 0; s < 4; ++s) {
    int m = (s < ns) ? g.nb[4 * c + s] : -1;
    nbm[s] = (m >= 0 && g.type[m] == 1) ? m : -1;
  }
  double a[6] = {0, 0, 0, 0, 0, 0};
  double itb = 0.0;
  double ab[4] = {0, 0, 0, 0};  // bars of the face coefficients per slot
  const double hn = rho * pow(lam / kPi, 0.5 * D);
  const double shc = 4.0 * (1.0 - g.pr) * lam * lam / (5.0 * rho);
  for (int k = lane; k < nv; k += 64) {
    const size_t o = (size_t)c * nv + k;
    const double vx = g.vx[k], vy = g.vy[k];
    const double xh = h1[o] - h0[o], xb = b1[o] - b0[o];
    const double ddb = -rh[o] * xh + (yh[o] - rh[o]) * (xsh[o] - xh) - rb[o] * xb + (yb[o] - rb[o]) * (xsb[o] - xb);
    itb += 0.5 * ddb;
    for (int s = 0; s < ns; ++s) {
      const double cf = micro_coef(mg, s, vx, vy);
      double t = 0.0;
      if (cf > 0.0) t = ddb;
      else if (cf < 0.0 && nbm[s] >= 0) {
        const int m = nbm[s];
        const size_t om = (size_t)m * nv + k;
        if (m < c) t = -(rh[o] * xsh[om] + rb[o] * xsb[om]);
        else t = -(yh[o] * (h1[om] - h0[om]) + yb[o] * (b1[om] - b0[om]));
      }
      ab[s] += t;
    }
    // residual: r = S - f/dt + (D + (f+ - f) / tau) / 2
    const double cx = vx - ux, cy = (D == 2) ? vy - uy : 0.0;
    const double c2 = cx * cx + cy * cy;
    const double H = hn * exp(-lam * c2);
    const double beta = (double)kNxi / (2.0 * lam);
    const double sq = shc * (cx * qx + cy * qy);
    const double hp = H + sq * (2.0 * lam * c2 - 2.0 - D) * H;
    const double bp = beta * H + sq * (2.0 * lam * c2 - D) * beta * H;
    Shb[o] = rh[o];
    Sbb[o] = rb[o];
    Dbh[o] = 0.5 * rh[o];
    Dbb[o] = 0.5 * rb[o];
    hbar[o] = xbh[o] + rh[o] * (-1.0 / dt - 0.5 * it);
    bbar[o] = xbb[o] + rb[o] * (-1.0 / dt - 0.5 * it);
    itb += 0.5 * (rh[o] * (hp - h0[o]) + rb[o] * (bp - b0[o]));
    const double eh = 0.5 * it * rh[o], eb = 0.5 * it * rb[o];
    eq_rev(g, rho, ux, uy, lam, qx, qy, vx, vy, eh, eb, eh, eb, a);
  }
  for (int i = 0; i < 6; ++i) a[i] = wave_sum(a[i]);
  itb = wave_sum(itb);
  for (int s = 0; s < ns; ++s) ab[s] = wave_sum(ab[s]);
  double dr, dl;
  itau_partials(g, rho, lam, dr, dl);
  if (g.mu_ref > 0.0) { a[0] += itb * dr; a[3] += itb * dl; }
  // q~ = heat flux of f about the velocity of W~
  const double qxb = a[4], qyb = a[5];
  double uxq = 0.0, uyq = 0.0;
  for (int k = lane; k < nv; k += 64) {
    const size_t o = (size_t)c * nv + k;
    double dh, db;
    heat_rev_k(D, g.wk[k], g.vx[k], g.vy[k], ux, uy, h0[o], b0[o], qxb, qyb, dh, db, uxq, uyq);
    hbar[o] += dh;
    bbar[o] += db;
  }
  const double uxb = a[1] + wave_sum(uxq);
  const double uyb = a[2] + wave_sum(uyq);
  double Wl[4] = {0, 0, 0, 0};
  prim_rev(D, kNxi, Wp + (size_t)c * nw, a[0], uxb, uyb, a[3], Wl);
  if (lane < nw) Wpb[(size_t)c * nw + lane] += Wl[lane];
  // face coefficient a = S/(2|Omega|) (v - U_f).n_out = A vx + B vy - C:
  // its U_f bar is -(A, B) a_bar, kept per (cell, slot) and added to the
  // faces by k_adj_slot_fold
  if (lane < ns) {
    const int s = lane;
    sbar[(size_t)(4 * c + s) * 2 + 0] = -mg[3 * s] * ab[s];
    sbar[(size_t)(4 * c + s) * 2 + 1] = -mg[3 * s + 1] * ab[s];
  }
}

// per face: the U_f bars of the micro coefficients of its field cells, the
// left cell's before the right one's
__global__ void k_adj_slot_fold(Dev g, const double* __restrict__ sbar, double* __restrict__ fbar) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= g.nface) return;
  const int L = g.fcell[2 * f], R = g.fcell[2 * f + 1];
  double ax = 0.0, ay = 0.0;
  for (int side = 0; side < 2; ++side) {
    const int c = side ? R : L;
    if (c < 0 || (side == 1 && R == L) || g.type[c] != 1) continue;
    for (int s = 0; s < 2 * kD; ++s)
      if (g.cf[4 * c + s] == f) {
        ax += sbar[(size_t)(4 * c + s) * 2 + 0];
        ay += sbar[(size_t)(4 * c + s) * 2 + 1];
      }
  }
  fbar[(size_t)f * 5 + 0] += ax;
  fbar[(size_t)f * 5 + 1] += ay;
}

// ------------------------------------------------------------------------
// macro LU-SGS reversed (Eq. dualTimeStepping_macro)
// ------------------------------------------------------------------------
// ALE Euler flux along n with mesh normal velocity un (D + N_xi = 3)
__device__ inline void euler_f(int D, const double* w, double nx, double ny, double un, double* o) {
  double vx = w[1] / w[0], vy = (D == 2) ? w[2] / w[0] : 0.0;
  double wE = w[D + 1];
  double p = 2.0 / 3.0 * (wE - 0.5 * w[0] * (vx * vx + vy * vy));
  double vn = vx * nx + ((D == 2) ? vy * ny : 0.0);
  double th = vn - un;
  o[0] = w[0] * th;
  o[1] = w[1] * th + p * nx;
  if (D == 2) { o[2] = w[2] * th + p * ny; o[3] = wE * th + p * vn; }
  else o[2] = wE * th + p * vn;
}

// Wb += (d F_E / d W)^T ab
__device__ inline void euler_vjp(int D, const double* w, double nx, double ny, double un, const double* ab,
                                 double* Wb) {
  const int E = D + 1;
  double rho = w[0];
  double vx = w[1] / rho, vy = (D == 2) ? w[2] / rho : 0.0;
  double p = 2.0 / 3.0 * (w[E] - 0.5 * rho * (vx * vx + vy * vy));
  double vn = vx * nx + ((D == 2) ? vy * ny : 0.0);
  double th = vn - un;
  double thb = 0.0;
  for (int m = 0; m <= E; ++m) { thb += ab[m] * w[m]; Wb[m] += ab[m] * th; }
  double pb = ab[1] * nx + ((D == 2) ? ab[2] * ny : 0.0) + ab[E] * vn;
  double vnb = thb + ab[E] * p;
  Wb[1] += vnb * nx / rho;
  if (D == 2) Wb[2] += vnb * ny / rho;
  Wb[0] += -vnb * vn / rho;
  const double k = 2.0 / 3.0;
  Wb[E] += k * pb;
  Wb[1] += -k * pb * vx;
  if (D == 2) Wb[2] += -k * pb * vy;
  Wb[0] += k * pb * 0.5 * (vx * vx + vy * vy);
}

// base bar of dW: the predictor W~ = W + dW (or W where W + dW is not a
// physical state: the solver keeps W there)
__global__ void k_adj_macro_init(Dev g, const double* __restrict__ W, const double* __restrict__ dW,
                                 const double* __restrict__ Wpb, double* __restrict__ Wbar,
                                 double* __restrict__ dWb) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= g.ncell) return;
  const int nw = kNw;
  bool upd = false;
  if (g.type[c] == 1) {
    double t[4] = {0, 0, 0, 0};
    for (int m = 0; m < nw; ++m) t[m] = W[(size_t)c * nw + m] + dW[(size_t)c * nw + m];
    upd = physical_state(kD, t);
  }
  for (int m = 0; m < nw; ++m) {
    double v = Wpb[(size_t)c * nw + m];
    Wbar[(size_t)c * nw + m] += v;
    dWb[(size_t)c * nw + m] = upd ? v : 0.0;
  }
}

// reverse of the two nonlinear sweeps, one workgroup per block, one thread
// per row; pass 1 (ascending hyperplanes) reverses the backward sweep,
// pass 2 (descending) the forward sweep
__global__ __launch_bounds__(512) void k_adj_macro_sweep(
    Dev g, const int* __restrict__ binfo, double dt, const double* __restrict__ W,
    const double* __restrict__ dWs, const double* __restrict__ dW, const double* __restrict__ gam,
    const double* __restrict__ dWb, double* __restrict__ abar, double* __restrict__ bbarm,
    double* __restrict__ dWsb, double* __restrict__ Rb, double* __restrict__ Dgb, double* __restrict__ gamb,
    double* __restrict__ Wbar, double* __restrict__ fbar) {
  const int blk = blockIdx.x;
  const int ni = binfo[8 * blk], nj = binfo[8 * blk + 1], c0 = binfo[8 * blk + 2];
  const int D = kD, nw = kNw, ns = 2 * D;
  const int nh = ni + nj - 1;
  for (int pass = 0; pass < 2; ++pass) {
    for (int it = 0; it < nh; ++it) {
      const int hp = (pass == 0) ? it : nh - 1 - it;
      for (int j = threadIdx.x; j < nj; j += blockDim.x) {
        const int i = hp - j;
        if (i < 0 || i >= ni) continue;
        const int n = c0 + i + ni * j;
        if (g.type[n] != 1) continue;
        const double ivol = 1.0 / g.vol[n];
        double sg = 0.0;
        for (int s = 0; s < ns; ++s) {
          int f = g.cf[4 * n + s];
          if (f >= 0) sg += g.fgeo[(size_t)f * 8 + 2] * gam[f];
        }
        const double Dg = 1.0 / g.dtp[n] + 1.0 / dt + 0.25 * ivol * sg;
        const double* Wn_ = W + (size_t)n * nw;
        const double* x = (pass == 0) ? dW + (size_t)n * nw : dWs + (size_t)n * nw;
        double base[4] = {0, 0, 0, 0}, Wl[4] = {0, 0, 0, 0}, acc[4] = {0, 0, 0, 0};
        for (int m = 0; m < nw; ++m) base[m] = (pass == 0) ? dWb[(size_t)n * nw + m] : dWsb[(size_t)n * nw + m];
        double Wt[4] = {0, 0, 0, 0};
        for (int m = 0; m < nw; ++m) Wt[m] = Wn_[m] + x[m];
        for (int s = 0; s < ns; ++s) {
          const int m_ = g.nb[4 * n + s];
          if (m_ < 0 || g.type[m_] != 1) continue;
          const int f = g.cf[4 * n + s];
          const double* fg = g.fgeo + (size_t)f * 8;
          const double S = fg[2];
          const double sig = (s & 1) ? 1.0 : -1.0;
          const double nx = sig * fg[0], ny = sig * fg[1];
          const double un = fg[3] * nx + fg[4] * ny;
          const bool lower = m_ < n;
          if (lower == (pass == 0)) {
            // the neighbour coupled this cell into its own sweep: gather its bar
            const double* am = ((pass == 0) ? abar : bbarm) + (size_t)m_ * nw;
            double v1[4] = {0, 0, 0, 0}, v0[4] = {0, 0, 0, 0};
            euler_vjp(D, Wt, -nx, -ny, -un, am, v1);
            euler_vjp(D, Wn_, -nx, -ny, -un, am, v0);
            double ax_ = 0.0;
            for (int m = 0; m < nw; ++m) {
              base[m] += S * (v1[m] - gam[f] * am[m]);
              Wl[m] += S * (v1[m] - v0[m]);
              ax_ += am[m] * x[m];
            }
            gamb[f] += -S * ax_;
            // un of the neighbour's normal is -un: F_E depends on it through -W
            fbar[(size_t)f * 5 + 0] += -S * ax_ * (-nx);
            fbar[(size_t)f * 5 + 1] += -S * ax_ * (-ny);
          } else if (pass == 0) {
            // this cell's own backward-sweep coupling (recomputed)
            const double* xm = dW + (size_t)m_ * nw;
            const double* Wm = W + (size_t)m_ * nw;
            double w1[4] = {0, 0, 0, 0}, e1[4], e0[4];
            for (int m = 0; m < nw; ++m) w1[m] = Wm[m] + xm[m];
            euler_f(D, w1, nx, ny, un, e1);
            euler_f(D, Wm, nx, ny, un, e0);
            for (int m = 0; m < nw; ++m) acc[m] += S * (e1[m] - e0[m]) - S * gam[f] * xm[m];
          }
        }
        const double ab = -0.25 * ivol / Dg;
        double dgb = 0.0;
        for (int m = 0; m < nw; ++m) {
          Wbar[(size_t)n * nw + m] += Wl[m];
          if (pass == 0) {
            abar[(size_t)n * nw + m] = ab * base[m];
            dWsb[(size_t)n * nw + m] = base[m];
            dgb += 0.25 * ivol * base[m] * acc[m] / (Dg * Dg);
          } else {
            bbarm[(size_t)n * nw + m] = ab * base[m];
            Rb[(size_t)n * nw + m] = base[m] / Dg;
            dgb += -base[m] * x[m] / Dg;
          }
        }
        Dgb[n] += dgb;
      }
      __syncthreads();
    }
  }
}

// residual bars to W and Wn; one thread per cell
__global__ void k_adj_macro_post(Dev g, double dt, const double* __restrict__ Rb, double* __restrict__ Wbar,
                                 double* __restrict__ Wnb) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= g.ncell) return;
  const int nw = kNw;
  if (g.type[c] != 1) return;
  for (int m = 0; m < nw; ++m) {
    double r = Rb[(size_t)c * nw + m];
    Wbar[(size_t)c * nw + m] -= r / dt;
    Wnb[(size_t)c * nw + m] += r / dt;
  }
}

// residual and diagonal bars to the faces' F, Fn and Gamma: one thread per
// face, its field cells in the order left, right
__global__ void k_adj_macro_face(Dev g, const double* __restrict__ Rb, const double* __restrict__ Dgb,
                                 double* __restrict__ Fbar, double* __restrict__ Fnb, double* __restrict__ gamb) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= g.nface) return;
  const int nw = kNw;
  const int L = g.fcell[2 * f], R = g.fcell[2 * f + 1];
  const double S = g.fgeo[(size_t)f * 8 + 2];
  for (int side = 0; side < 2; ++side) {
    const int c = side ? R : L;
    if (c < 0 || (side == 1 && R == L) || g.type[c] != 1) continue;
    const double ivol = 1.0 / g.vol[c];
    for (int s = 0; s < 2 * kD; ++s) {
      if (g.cf[4 * c + s] != f) continue;
      const double sig = (s & 1) ? 1.0 : -1.0;
      for (int m = 0; m < nw; ++m) {
        const double v = -0.5 * ivol * sig * S * Rb[(size_t)c * nw + m];
        acc_add(Fbar + (size_t)f * nw + m, v);
        acc_add(Fnb + (size_t)f * nw + m, v);
      }
      acc_add(gamb + f, 0.25 * ivol * S * Dgb[c]);
    }
  }
}

// spectral radius Gamma of a face reversed: one thread per face
__global__ void k_adj_gamma(Dev g, const int* __restrict__ items, int nitems, const double* __restrict__ W,
                            const double* __restrict__ gamb, double* __restrict__ Wbar, double* __restrict__ fbar) {
  const int slot = blockIdx.x * blockDim.x + threadIdx.x;
  if (slot >= nitems) return;
  const int f = items[slot];
  const double gb = gamb[f];
  if (gb == 0.0) return;
  const int D = kD, nw = kNw;
  const int L = g.fcell[2 * f], R = g.fcell[2 * f + 1];
  const double* fg = g.fgeo + (size_t)f * 8;
  const double nx = fg[0], ny = fg[1];
  const double gma = (double)(D + kNxi + 2) / (double)(D + kNxi);
  auto side = [&](int code, int inner, double wgt_u, double wgt_a, double thb) {
    const double* w;
    int tgt;
    if (code >= 0) { w = W + (size_t)code * nw; tgt = code; }
    else if (code == kNbFar) return;
    else { w = W + (size_t)inner * nw; tgt = inner; }
    double rho, ux, uy, lam;
    prim_d(D, kNxi, w, rho, ux, uy, lam);
    double a = sqrt(gma * 0.5 / lam);
    double lb = -wgt_a * gb * a / (2.0 * lam);
    double Wl[4] = {0, 0, 0, 0};
    prim_rev(D, kNxi, w, 0.0, wgt_u * thb * nx, wgt_u * thb * ny, lb, Wl);
    for (int m = 0; m < nw; ++m) acc_add(Wbar + (size_t)tgt * nw + m, Wl[m]);
  };
  double thv;
  if (L == kNbWall || R == kNbWall) {
    int c = (L == kNbWall) ? R : L;
    if (c < 0) return;
    double rho, ux, uy, lam;
    prim_d(D, kNxi, W + (size_t)c * nw, rho, ux, uy, lam);
    thv = (ux - fg[3]) * nx + (uy - fg[4]) * ny;
    double thb = gb * ((thv < 0.0) ? -1.0 : 1.0);
    side(c, c, 1.0, 1.0, thb);
    fbar[(size_t)f * 5 + 0] += -thb * nx;
    fbar[(size_t)f * 5 + 1] += -thb * ny;
    return;
  }
  int inner = (L >= 0) ? L : R;
  if (inner < 0) return;
  auto vel = [&](int code, double& ux, double& uy) {
    const double* w = (code >= 0) ? W + (size_t)code * nw : ((code == kNbFar) ? g.winf : W + (size_t)inner * nw);
    ux = w[1] / w[0];
    uy = (D == 2) ? w[2] / w[0] : 0.0;
  };
  double u1, v1, u2, v2;
  vel(L, u1, v1);
  vel(R, u2, v2);
  thv = (0.5 * (u1 + u2) - fg[3]) * nx + (0.5 * (v1 + v2) - fg[4]) * ny;
  double thb = gb * ((thv < 0.0) ? -1.0 : 1.0);
  side(L, inner, 0.5, 0.5, thb);
  side(R, inner, 0.5, 0.5, thb);
  fbar[(size_t)f * 5 + 0] += -thb * nx;
  fbar[(size_t)f * 5 + 1] += -thb * ny;
}

// ------------------------------------------------------------------------
// Steps 1-2 source S = f/dt + (D + (f+ - f)/tau)/2 reversed (one wavefront
// per cell): bars of f, of the divergence D and of (W, q) through f+ and tau
// ------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_adj_source(Dev g, double dt, const double* __restrict__ crec,
                                                    const double* __restrict__ W, const double* __restrict__ h,
                                                    const double* __restrict__ b, const double* __restrict__ Shb,
                                                    const double* __restrict__ Sbb, double* __restrict__ hbar,
                                                    double* __restrict__ bbar, double* __restrict__ Dbh,
                                                    double* __restrict__ Dbb, double* __restrict__ Wbar,
                                                    double* __restrict__ qbar) {
  const int c = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (c >= g.ncell) return;
  const int D = kD, nv = g.nv, nw = kNw;
  if (g.type[c] != 1) {
    for (int k = lane; k < nv; k += 64) { Dbh[(size_t)c * nv + k] = 0.0; Dbb[(size_t)c * nv + k] = 0.0; }
    return;
  }
  const double* r = crec + (size_t)c * NCREC;
  const double rho = r[C_RHO], ux = r[C_UX], uy = r[C_UY], lam = r[C_LAM], qx = r[C_QX], qy = r[C_QY];
  const double it = r[C_ITAU];
  const double hn = rho * pow(lam / kPi, 0.5 * D);
  const double shc = 4.0 * (1.0 - g.pr) * lam * lam / (5.0 * rho);
  double a[6] = {0, 0, 0, 0, 0, 0};
  double itb = 0.0;
  for (int k = lane; k < nv; k += 64) {
    const size_t o = (size_t)c * nv + k;
    const double vx = g.vx[k], vy = g.vy[k];
    const double sh = Shb[o], sb = Sbb[o];
    const double cx = vx - ux, cy = (D == 2) ? vy - uy : 0.0;
    const double c2 = cx * cx + cy * cy;
    const double H = hn * exp(-lam * c2);
    const double beta = (double)kNxi / (2.0 * lam);
    const double sq = shc * (cx * qx + cy * qy);
    const double hp = H + sq * (2.0 * lam * c2 - 2.0 - D) * H;
    const double bp = beta * H + sq * (2.0 * lam * c2 - D) * beta * H;
    hbar[o] += sh * (1.0 / dt - 0.5 * it);
    bbar[o] += sb * (1.0 / dt - 0.5 * it);
    Dbh[o] = 0.5 * sh;
    Dbb[o] = 0.5 * sb;
    itb += 0.5 * (sh * (hp - h[o]) + sb * (bp - b[o]));
    eq_rev(g, rho, ux, uy, lam, qx, qy, vx, vy, 0.5 * it * sh, 0.5 * it * sb, 0.5 * it * sh, 0.5 * it * sb, a);
  }
  for (int i = 0; i < 6; ++i) a[i] = wave_sum(a[i]);
  itb = wave_sum(itb);
  double dr, dl;
  itau_partials(g, rho, lam, dr, dl);
  if (g.mu_ref > 0.0) { a[0] += itb * dr; a[3] += itb * dl; }
  double Wl[4] = {0, 0, 0, 0};
  prim_rev(D, kNxi, W + (size_t)c * nw, a[0], a[1], a[2], a[3], Wl);
  if (lane < nw) acc_add(Wbar + (size_t)c * nw + lane, Wl[lane]);
  if (lane == 0) {
    acc_add(qbar + (size_t)c * D, a[4]);
    if (D == 2) acc_add(qbar + (size_t)c * D + 1, a[5]);
  }
}

// ------------------------------------------------------------------------
// overset interpolation reversed (Sec. 3.2): the bars of the rows' target
// cells move to their donors and the targets' bars become zero; one
// wavefront per row (donors are never targets of the same call)
// ------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_adj_interp(Dev g, const int* __restrict__ items, int nitems,
                                                    const int* __restrict__ rec, const int* __restrict__ ptr,
                                                    const int* __restrict__ don, const double* __restrict__ wt,
                                                    double* __restrict__ hbar, double* __restrict__ bbar,
                                                    double* __restrict__ Wbar, double* __restrict__ qbar) {
  const int slot = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (slot >= nitems) return;
  const int r = items[slot];
  const int c = rec[r], p0 = ptr[r], p1 = ptr[r + 1];
  for (int k = lane; k < g.nv; k += 64) {
    const size_t o = (size_t)c * g.nv + k;
    const double vh = hbar[o], vb = bbar[o];
    for (int p = p0; p < p1; ++p) {
      acc_add(hbar + (size_t)don[p] * g.nv + k, wt[p] * vh);
      acc_add(bbar + (size_t)don[p] * g.nv + k, wt[p] * vb);
    }
    hbar[o] = 0.0;
    bbar[o] = 0.0;
  }
  if (lane < kNw) {
    const double v = Wbar[(size_t)c * kNw + lane];
    for (int p = p0; p < p1; ++p) acc_add(Wbar + (size_t)don[p] * kNw + lane, wt[p] * v);
    Wbar[(size_t)c * kNw + lane] = 0.0;
  }
  if (lane >= 8 && lane < 8 + kD) {
    const int m = lane - 8;
    const double v = qbar[(size_t)c * kD + m];
    for (int p = p0; p < p1; ++p) acc_add(qbar + (size_t)don[p] * kD + m, wt[p] * v);
    qbar[(size_t)c * kD + m] = 0.0;
  }
}

// ------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------
static inline unsigned nblk(size_t n, unsigned t) { return (unsigned)((n + t - 1) / t); }

// one launch per colour of an order; `wave` items per block of `threads`
template <typename F>
static void per_colour(const Order& o, int wave, unsigned threads, F launch) {
  for (int i = 0; i < o.ncolour; ++i) {
    const int n = o.off[i + 1] - o.off[i];
    if (n > 0) launch(dim3(nblk(n, wave)), dim3(threads), o.items + o.off[i], n);
  }
}

// threads of a face block: a wavefront per 512 velocities, at most
// kFaceWaves
static unsigned face_threads(int nv) {
  const int w = std::min(kFaceWaves, std::max(1, (nv + 511) / 512));
  return 64u * (unsigned)w;
}

void adj_flux(const Dev& g, const Order& faces, const Order& walls, const Order& cells, double dts,
              const double* h, const double* b, const double* W, const double* q, const double* gW,
              const double* rec, const double* Dbh, const double* Dbb, const double* Fb, double* hbar, double* bbar,
              double* Wbar, double* qbar, double* gWbar, double* fbar, double* fsc, hipStream_t st) {
  const unsigned nt = face_threads(g.nv);
  per_colour(faces, 1, nt, [&](dim3, dim3 bl, const int* it, int n) {
    for (int o = 0; o < n; o += kFaceBlocks) {
      const int m = std::min(n - o, kFaceBlocks);
      hipLaunchKernelGGL(k_adj_face, dim3((unsigned)m), bl, 0, st, g, it + o, m, dts, h, b, gW, rec, Dbh, Dbb, Fb,
                         hbar, bbar, gWbar, fbar, fsc);
    }
  });
  per_colour(walls, 1, nt, [&](dim3 gr, dim3 bl, const int* it, int n) {
    hipLaunchKernelGGL(k_adj_wall, gr, bl, 0, st, g, it, n, dts, h, b, W, q, gW, Dbh, Dbb, Fb, hbar, bbar, Wbar,
                       qbar, gWbar, fbar);
  });
  per_colour(cells, 128, 128, [&](dim3 gr, dim3 bl, const int* it, int n) {
    hipLaunchKernelGGL(k_adj_gradW, gr, bl, 0, st, g, it, n, W, gWbar, Wbar);
  });
}

void adj_step7(const Dev& g, const double* h1, const double* b1, const double* W1, const double* Wp,
               const double* W1b, const double* q1b, double* hb, double* bb, double* Wpb, hipStream_t st) {
  hipLaunchKernelGGL(k_adj_step7, dim3(nblk(g.ncell, 4)), dim3(256), 0, st, g, h1, b1, W1, Wp, W1b, q1b, hb, bb,
                     Wpb);
}

void adj_micro(const Dev& g, const int* binfo, int nblock, double dt, const double* crec, const double* Wp,
               const double* h0, const double* b0, const double* h1, const double* b1, const double* xsh,
               const double* xsb, const double* xbh, const double* xbb, double* yh, double* yb, double* rh,
               double* rb, double* hbar, double* bbar, double* Shb, double* Sbb, double* Dbh, double* Dbb,
               double* Wpb, double* sbar, double* fbar, hipStream_t st) {
  dim3 grid(nblock, nblk(g.nv, 16));
  hipLaunchKernelGGL(k_adj_micro_sweep<0>, grid, dim3(1024), 0, st, g, binfo, crec, xbh, xbb, yh, yb);
  hipLaunchKernelGGL(k_adj_micro_sweep<1>, grid, dim3(1024), 0, st, g, binfo, crec, (const double*)yh,
                     (const double*)yb, rh, rb);
  hipLaunchKernelGGL(k_adj_micro_coef, dim3(nblk(g.ncell, 4)), dim3(256), 0, st, g, dt, crec, Wp, h0, b0, h1, b1,
                     xsh, xsb, (const double*)yh, (const double*)yb, (const double*)rh, (const double*)rb, xbh, xbb,
                     hbar, bbar, Shb, Sbb, Dbh, Dbb, Wpb, sbar);
  if (g.nface > 0)
    hipLaunchKernelGGL(k_adj_slot_fold, dim3(nblk(g.nface, 128)), dim3(128), 0, st, g, (const double*)sbar, fbar);
}

void adj_macro(const Dev& g, const Order& faces, const Order& walls, const int* binfo, int nblock, double dt,
               const double* W, const double* dWs, const double* dW, const double* gam, const double* Wpb,
               double* dWb, double* abar, double* bbarm, double* dWsb, double* Rb, double* Dgb, double* gamb,
               double* Wbar, double* Wnb, double* Fbar, double* Fnb, double* fbar, hipStream_t st) {
  hipLaunchKernelGGL(k_adj_macro_init, dim3(nblk(g.ncell, 128)), dim3(128), 0, st, g, W, dW, Wpb, Wbar, dWb);
  hipLaunchKernelGGL(k_adj_macro_sweep, dim3(nblock), dim3(512), 0, st, g, binfo, dt, W, dWs, dW, gam,
                     (const double*)dWb, abar, bbarm, dWsb, Rb, Dgb, gamb, Wbar, fbar);
  hipLaunchKernelGGL(k_adj_macro_post, dim3(nblk(g.ncell, 128)), dim3(128), 0, st, g, dt, (const double*)Rb, Wbar,
                     Wnb);
  if (g.nface > 0)
    hipLaunchKernelGGL(k_adj_macro_face, dim3(nblk(g.nface, 128)), dim3(128), 0, st, g, (const double*)Rb,
                       (const double*)Dgb, Fbar, Fnb, gamb);
  for (const Order* o : {&faces, &walls})
    per_colour(*o, 128, 128, [&](dim3 gr, dim3 bl, const int* it, int n) {
      hipLaunchKernelGGL(k_adj_gamma, gr, bl, 0, st, g, it, n, W, (const double*)gamb, Wbar, fbar);
    });
}

void adj_source(const Dev& g, double dt, const double* crec, const double* W, const double* h, const double* b,
                const double* Shb, const double* Sbb, double* hbar, double* bbar, double* Dbh, double* Dbb,
                double* Wbar, double* qbar, hipStream_t st) {
  hipLaunchKernelGGL(k_adj_source, dim3(nblk(g.ncell, 4)), dim3(256), 0, st, g, dt, crec, W, h, b, Shb, Sbb, hbar,
                     bbar, Dbh, Dbb, Wbar, qbar);
}

void adj_interp(const Dev& g, const Order& rows, const int* rec, const int* ptr, const int* don, const double* w,
                double* hbar, double* bbar, double* Wbar, double* qbar, hipStream_t st) {
  per_colour(rows, 4, 256, [&](dim3 gr, dim3 bl, const int* it, int n) {
    hipLaunchKernelGGL(k_adj_interp, gr, bl, 0, st, g, it, n, rec, ptr, don, w, hbar, bbar, Wbar, qbar);
  });
}

}  // namespace ugks
