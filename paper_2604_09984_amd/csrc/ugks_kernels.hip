// HIP kernels (gfx950, wave64) of one dual-time pseudo-iteration of the
// implicit unsteady UGKS on moving overset structured meshes.
//
// Layout: h, b [ncell][nv] velocity innermost, so a wavefront whose lanes are
// 64 consecutive velocities reads 64 consecutive values of one cell.
// Velocity reductions are wavefront shuffles accumulated in double.
#include "ugks_kernels.h"

namespace ugks {

// ------------------------------------------------------------------------
// normal relative velocity; no contraction, so that exact zeros (an upwind
// tie) are reproduced bit for bit
// ------------------------------------------------------------------------
__device__ __attribute__((noinline)) double wnorm(double vx, double vy, double ux, double uy,
                                                  double nx, double ny) {
#pragma clang fp contract(off)
  return (vx - ux) * nx + (vy - uy) * ny;
}

// limited slope per unit index along dir (van Leer; one-sided beside a wall;
// zero beside a hole / fringe)
template <class T>
__device__ inline double index_slope(const Dev& g, const T* __restrict__ f, const T* __restrict__ finf,
                                     int c, int dir, int k, double v0) {
  int lo = g.nb[4 * c + 2 * dir], hi = g.nb[4 * c + 2 * dir + 1];
  if (lo == kNbMiss || hi == kNbMiss) return 0.0;
  auto val = [&](int code) -> double {
    if (code >= 0) return (double)f[(size_t)code * g.nv + k];
    if (code == kNbFar) return (double)finf[k];
    return v0;  // copy ghost
  };
  if (lo == kNbWall && hi == kNbWall) return 0.0;
  if (lo == kNbWall) return val(hi) - v0;
  if (hi == kNbWall) return v0 - val(lo);
  double s1 = v0 - val(lo), s2 = val(hi) - v0;
  if (s1 * s2 <= 0.0) return 0.0;
  return (s1 * fabs(s2) + fabs(s1) * s2) / (fabs(s1) + fabs(s2));
}

// reconstruction of cell c at the face in its slot: face value and gradient
template <class T>
__device__ inline void recon(const Dev& g, const T* __restrict__ f, const T* __restrict__ finf, int c,
                             int slot, int k, double& val, double& gx, double& gy) {
  double v0 = (double)f[(size_t)c * g.nv + k];
  double si = index_slope(g, f, finf, c, 0, k, v0);
  double sj = (g.dim == 2) ? index_slope(g, f, finf, c, 1, k, v0) : 0.0;
  const double* G = g.G + 4 * c;
  gx = G[0] * si + G[1] * sj;
  gy = (g.dim == 2) ? G[2] * si + G[3] * sj : 0.0;
  val = v0 + gx * g.cdx[8 * c + 2 * slot] + gy * g.cdx[8 * c + 2 * slot + 1];
}

// side data of face f seen from cell c in slot s: the other side
template <class T>
__device__ inline void other_side(const Dev& g, const T* __restrict__ f, const T* __restrict__ finf,
                                  int c, int s, int o, int k, double& val, double& gx, double& gy) {
  if (o >= 0) {
    recon(g, f, finf, o, s ^ 1, k, val, gx, gy);
  } else {
    val = (o == kNbFar) ? (double)finf[k] : (double)f[(size_t)c * g.nv + k];
    gx = gy = 0.0;
  }
}

// interface distribution integrated over dt_s and divided by dt_s
// (Eq. fullSolution with the coefficient integrals) for h (m = 0) and b
// (m = 1), computed in type C
template <class C>
struct FaceEq {
  C rho, ux, uy, lam, qx, qy, hn, sh, ax[4], ay[4], at[4], t[5];
  __device__ void load(const double* r) {
    rho = (C)r[R_RHO]; ux = (C)r[R_UX]; uy = (C)r[R_UY]; lam = (C)r[R_LAM];
    qx = (C)r[R_QX]; qy = (C)r[R_QY]; hn = (C)r[R_HN]; sh = (C)r[R_SH];
    for (int m = 0; m < 4; ++m) { ax[m] = (C)r[R_AX + m]; ay[m] = (C)r[R_AY + m]; at[m] = (C)r[R_AT + m]; }
    for (int m = 0; m < 5; ++m) t[m] = (C)r[R_T1 + m];
  }
};

template <class C>
__device__ inline C expo(C x);
template <>
__device__ inline double expo<double>(double x) { return exp(x); }
template <>
__device__ inline float expo<float>(float x) { return expf(x); }

template <class C>
__device__ inline void interface_avg(const FaceEq<C>& e, int dim, int nxi, C vx, C vy, C wx, C wy,
                                     C fh, C fb, C ghx, C ghy, C gbx, C gby, C& Ih, C& Ib) {
  C cx = vx - e.ux, cy = (dim == 2) ? vy - e.uy : C(0);
  C c2 = cx * cx + cy * cy;
  C H = e.hn * expo<C>(-e.lam * c2);
  C rt = C(0.5) / e.lam;
  C B = C(nxi) * rt * H;
  C s = e.sh * (cx * e.qx + cy * e.qy);
  C twol = C(2) * e.lam * c2;
  C Hp = s * (twol - C(2) - C(dim)) * H;
  C Bp = s * (twol - C(dim)) * C(nxi) * rt * H;
  C v2 = vx * vx + ((dim == 2) ? vy * vy : C(0));
  C eh = C(0.5) * (v2 + C(nxi) * rt);       // energy factor of (a.psi) for h
  C eb = C(0.5) * (v2 + C(nxi + 2) * rt);   // for b
  int E = dim + 1;
  C pax = e.ax[0] + e.ax[1] * vx + ((dim == 2) ? e.ax[2] * vy : C(0));
  C pay = e.ay[0] + e.ay[1] * vx + ((dim == 2) ? e.ay[2] * vy : C(0));
  C pat = e.at[0] + e.at[1] * vx + ((dim == 2) ? e.at[2] * vy : C(0));
  C wah = wx * (pax + e.ax[E] * eh) + wy * (pay + e.ay[E] * eh);
  C wab = wx * (pax + e.ax[E] * eb) + wy * (pay + e.ay[E] * eb);
  C ath = pat + e.at[E] * eh, atb = pat + e.at[E] * eb;
  Ih = e.t[0] * fh + e.t[1] * (wx * ghx + wy * ghy) + e.t[2] * (H + Hp) + e.t[3] * wah * H + e.t[4] * ath * H;
  Ib = e.t[0] * fb + e.t[1] * (wx * gbx + wy * gby) + e.t[2] * (B + Bp) + e.t[3] * wab * B + e.t[4] * atb * B;
}

// ------------------------------------------------------------------------
// cell gradients of W (limited, physical): gW[cell][2][nw]
// ------------------------------------------------------------------------
__global__ void k_gradW(Dev g, const double* __restrict__ W, double* __restrict__ gW) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= g.ncell) return;
  double* o = gW + (size_t)c * 8;
  for (int m = 0; m < 8; ++m) o[m] = 0.0;
  if (g.type[c] == 0) return;
  for (int m = 0; m < g.nw; ++m) {
    double v0 = W[(size_t)c * g.nw + m];
    double s[2] = {0.0, 0.0};
    for (int dir = 0; dir < g.dim; ++dir) {
      int lo = g.nb[4 * c + 2 * dir], hi = g.nb[4 * c + 2 * dir + 1];
      if (lo == kNbMiss || hi == kNbMiss) continue;
      auto val = [&](int code) -> double {
        if (code >= 0) return W[(size_t)code * g.nw + m];
        if (code == kNbFar) return g.winf[m];
        return v0;
      };
      if (lo == kNbWall && hi == kNbWall) continue;
      if (lo == kNbWall) { s[dir] = val(hi) - v0; continue; }
      if (hi == kNbWall) { s[dir] = v0 - val(lo); continue; }
      double s1 = v0 - val(lo), s2 = val(hi) - v0;
      s[dir] = (s1 * s2 <= 0.0) ? 0.0 : (s1 * fabs(s2) + fabs(s1) * s2) / (fabs(s1) + fabs(s2));
    }
    const double* G = g.G + 4 * c;
    o[m] = G[0] * s[0] + G[1] * s[1];
    o[g.nw + m] = (g.dim == 2) ? G[2] * s[0] + G[3] * s[1] : 0.0;
  }
}

// ------------------------------------------------------------------------
// wall incident state of every active wall face (one-sided data of the
// interior cell): record fields R_RHO..R_T1, wall parameters, sign
// ------------------------------------------------------------------------
__global__ void k_wallprep(Dev g, double dts, const double* __restrict__ W, const double* __restrict__ q,
                           const double* __restrict__ gW, double* __restrict__ rec) {
  int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= g.nface) return;
  int L = g.fcell[2 * f], R = g.fcell[2 * f + 1];
  if (L != kNbWall && R != kNbWall) return;
  double* r = rec + (size_t)f * NREC;
  for (int m = 0; m < NREC; ++m) r[m] = 0.0;
  int c = (L == kNbWall) ? R : L;
  if (c < 0 || g.type[c] != 1) return;
  int dir = 0;
  for (int s = 0; s < 4; ++s) if (g.cf[4 * c + s] == f) dir = s;
  const double* fg = g.fgeo + (size_t)f * 8;
  int nw = g.nw;
  double Win[4];
  const double* gw = gW + (size_t)c * 8;
  double dx = g.cdx[8 * c + 2 * dir], dy = g.cdx[8 * c + 2 * dir + 1];
  for (int m = 0; m < nw; ++m) Win[m] = W[(size_t)c * nw + m] + gw[m] * dx + gw[nw + m] * dy;
  double rho, ux, uy, lam;
  prim_of(g, Win, rho, ux, uy, lam);
  r[R_RHO] = rho; r[R_UX] = ux; r[R_UY] = uy; r[R_LAM] = lam;
  r[R_QX] = q[(size_t)c * g.dim];
  r[R_QY] = (g.dim == 2) ? q[(size_t)c * g.dim + 1] : 0.0;
  r[R_HN] = rho * pow(lam / kPi, 0.5 * g.dim);
  r[R_SH] = 4.0 * (1.0 - g.pr) * lam * lam / (5.0 * rho);
  expansion(g.dim, rho, ux, uy, lam, fg[3], fg[4], gw, r + R_AX, r + R_AY, r + R_AT);
  double tq[5];
  time_integrals(dts, inv_tau_of(g, rho, lam), tq);
  for (int m = 0; m < 5; ++m) r[R_T1 + m] = tq[m] / dts;
  r[R_ACT] = 1.0;
  r[R_LAMW] = 0.5 / fg[7];
  r[R_HWN] = pow(r[R_LAMW] / kPi, 0.5 * g.dim);
  r[R_VWX] = fg[5];
  r[R_VWY] = fg[6];
  r[R_SGN] = (R == kNbWall) ? 1.0 : -1.0;
}

// ------------------------------------------------------------------------
// face equilibrium: one wavefront per cell, lanes over velocities; the cell
// reduces the faces it owns (its high faces, and low faces on a block
// boundary) and writes their records
// ------------------------------------------------------------------------
__device__ inline bool owns(const Dev& g, int c, int s, int f) {
  if (f < 0 || !g.fact[f]) return false;
  int other = g.fcell[2 * f + ((s & 1) ? 1 : 0)];
  return (s & 1) || other < 0;
}

template <class T>
__global__ __launch_bounds__(256) void k_face_eq(Dev g, double dts, const T* __restrict__ h,
                                                 const T* __restrict__ b, const double* __restrict__ W,
                                                 const double* __restrict__ gW, double* __restrict__ rec) {
  int c = blockIdx.x * 4 + (threadIdx.x >> 6);
  int lane = threadIdx.x & 63;
  if (c >= g.ncell || g.type[c] == 0) return;
  const T* hinf = (const T*)g.finf_h;
  const T* binf = (const T*)g.finf_b;
  int nw = g.nw;
  for (int s = 0; s < 2 * g.dim; ++s) {
    int f = g.cf[4 * c + s];
    if (!owns(g, c, s, f)) continue;
    int o = g.fcell[2 * f + ((s & 1) ? 1 : 0)];
    const double* fg = g.fgeo + (size_t)f * 8;
    double nx = fg[0], ny = fg[1], ufx = fg[3], ufy = fg[4];
    double* r = rec + (size_t)f * NREC;
    if (o == kNbWall) {
      // wall density from zero net mass flux (Eq. maxWalldes)
      if (g.type[c] != 1) continue;
      FaceEq<double> e;
      e.load(r);
      double sg = r[R_SGN], nwx = sg * nx, nwy = sg * ny;
      double lw = r[R_LAMW], hwn = r[R_HWN], vwx = r[R_VWX], vwy = r[R_VWY];
      double num = 0.0, den = 0.0;
      for (int k = lane; k < g.nv; k += 64) {
        double vx = g.vx[k], vy = g.vy[k];
        double wn = wnorm(vx, vy, ufx, ufy, nwx, nwy);
        if (wn > 0.0) {
          double fh, ghx, ghy, fb, gbx, gby;
          recon(g, h, hinf, c, s, k, fh, ghx, ghy);
          recon(g, b, binf, c, s, k, fb, gbx, gby);
          double Ih, Ib;
          interface_avg<double>(e, g.dim, g.nxi, vx, vy, vx - ufx, vy - ufy, fh, fb, ghx, ghy, gbx, gby, Ih, Ib);
          num += g.wk[k] * wn * Ih;
        } else if (wn < 0.0) {
          double cx = vx - vwx, cy = (g.dim == 2) ? vy - vwy : 0.0;
          den += g.wk[k] * wn * hwn * exp(-lw * (cx * cx + cy * cy));
        }
      }
      num = wave_sum(num);
      den = wave_sum(den);
      if (lane == 0) r[R_RHOW] = -num / den;
      continue;
    }
    // moments of the upwind interface data about the shift s = mean velocity
    int Lc = (s & 1) ? c : o, Rc = (s & 1) ? o : c;
    double sx, sy;
    {
      double r1, u1, v1, l1, r2, u2, v2, l2;
      auto Wof = [&](int code, double* out) {
        if (code >= 0) for (int m = 0; m < nw; ++m) out[m] = W[(size_t)code * nw + m];
        else if (code == kNbFar) for (int m = 0; m < nw; ++m) out[m] = g.winf[m];
        else for (int m = 0; m < nw; ++m) out[m] = W[(size_t)c * nw + m];
      };
      double WL[4], WR[4];
      Wof(Lc, WL);
      Wof(Rc, WR);
      prim_of(g, WL, r1, u1, v1, l1);
      prim_of(g, WR, r2, u2, v2, l2);
      sx = 0.5 * (u1 + u2);
      sy = 0.5 * (v1 + v2);
    }
    double m0 = 0, m1x = 0, m1y = 0, m2 = 0, pxx = 0, pxy = 0, pyy = 0, m3x = 0, m3y = 0;
    for (int k = lane; k < g.nv; k += 64) {
      double vx = g.vx[k], vy = g.vy[k];
      double wn = wnorm(vx, vy, ufx, ufy, nx, ny);
      double hc, bc, ho, bo, t0, t1;
      recon(g, h, hinf, c, s, k, hc, t0, t1);
      recon(g, b, binf, c, s, k, bc, t0, t1);
      other_side(g, h, hinf, c, s, o, k, ho, t0, t1);
      other_side(g, b, binf, c, s, o, k, bo, t0, t1);
      double hl = (s & 1) ? hc : ho, hr = (s & 1) ? ho : hc;
      double bl = (s & 1) ? bc : bo, br = (s & 1) ? bo : bc;
      double fh, fb;
      if (wn > 0.0) { fh = hl; fb = bl; }
      else if (wn < 0.0) { fh = hr; fb = br; }
      else { fh = 0.5 * (hl + hr); fb = 0.5 * (bl + br); }
      double w = g.wk[k];
      double cx = vx - sx, cy = (g.dim == 2) ? vy - sy : 0.0;
      double c2 = cx * cx + cy * cy;
      double e = c2 * fh + fb;
      m0 += w * fh;
      m1x += w * cx * fh;
      m1y += w * cy * fh;
      m2 += w * e;
      pxx += w * cx * cx * fh;
      pxy += w * cx * cy * fh;
      pyy += w * cy * cy * fh;
      m3x += w * cx * e;
      m3y += w * cy * e;
    }
    m0 = wave_sum(m0); m1x = wave_sum(m1x); m1y = wave_sum(m1y); m2 = wave_sum(m2);
    pxx = wave_sum(pxx); pxy = wave_sum(pxy); pyy = wave_sum(pyy);
    m3x = wave_sum(m3x); m3y = wave_sum(m3y);
    if (lane != 0) continue;
    // face state from the shifted moments
    double rho = m0;
    double dx = m1x / m0, dy = m1y / m0;
    double ux = sx + dx, uy = sy + dy;
    double eint = 0.5 * (m2 - (m1x * m1x + m1y * m1y) / m0);
    double lam = 0.25 * (double)(g.dim + g.nxi) * rho / eint;
    // heat flux about the face velocity: 2q = m3 - 2 P d - d m2 + 2 m0 |d|^2 d
    double dd = dx * dx + dy * dy;
    double qx = 0.5 * (m3x - 2.0 * (pxx * dx + pxy * dy) - dx * m2 + 2.0 * m0 * dd * dx);
    double qy = 0.5 * (m3y - 2.0 * (pxy * dx + pyy * dy) - dy * m2 + 2.0 * m0 * dd * dy);
    if (g.dim == 1) qy = 0.0;
    r[R_RHO] = rho; r[R_UX] = ux; r[R_UY] = uy; r[R_LAM] = lam; r[R_QX] = qx; r[R_QY] = qy;
    r[R_HN] = rho * pow(lam / kPi, 0.5 * g.dim);
    r[R_SH] = 4.0 * (1.0 - g.pr) * lam * lam / (5.0 * rho);
    double dW[8];
    for (int m = 0; m < 2 * nw; ++m) {
      double gl = (Lc >= 0) ? gW[(size_t)Lc * 8 + m] : 0.0;
      double gr = (Rc >= 0) ? gW[(size_t)Rc * 8 + m] : 0.0;
      dW[m] = 0.5 * (gl + gr);
    }
    expansion(g.dim, rho, ux, uy, lam, ufx, ufy, dW, r + R_AX, r + R_AY, r + R_AT);
    double tq[5];
    time_integrals(dts, inv_tau_of(g, rho, lam), tq);
    for (int m = 0; m < 5; ++m) r[R_T1 + m] = tq[m] / dts;
    r[R_ACT] = 1.0;
  }
}

// ------------------------------------------------------------------------
// flux: one wavefront per cell; divergence D of field cells, macro flux of
// the faces the cell owns (wall faces also give the wall output)
// ------------------------------------------------------------------------
template <class T, class C>
__global__ __launch_bounds__(256) void k_flux(Dev g, const T* __restrict__ h, const T* __restrict__ b,
                                              const double* __restrict__ rec, T* __restrict__ Dh,
                                              T* __restrict__ Db, double* __restrict__ F,
                                              double* __restrict__ wall) {
  int c = blockIdx.x * 4 + (threadIdx.x >> 6);
  int lane = threadIdx.x & 63;
  if (c >= g.ncell || g.type[c] == 0) return;
  const T* hinf = (const T*)g.finf_h;
  const T* binf = (const T*)g.finf_b;
  bool field = (g.type[c] == 1);
  double ivol = 1.0 / g.vol[c];
  int nw = g.nw;
  double acc[4][4];
  for (int s = 0; s < 4; ++s) for (int m = 0; m < 4; ++m) acc[s][m] = 0.0;
  for (int k0 = 0; k0 < g.nv; k0 += 64) {
    int k = k0 + lane;
    bool kin = k < g.nv;
    int kk = kin ? k : 0;
    double vx = g.vx[kk], vy = g.vy[kk], wk = kin ? g.wk[kk] : 0.0;
    C dh = 0, db = 0;
    for (int s = 0; s < 2 * g.dim; ++s) {
      int f = g.cf[4 * c + s];
      if (f < 0 || !g.fact[f]) continue;
      bool own = owns(g, c, s, f);
      if (!field && !own) continue;
      const double* r = rec + (size_t)f * NREC;
      const double* fg = g.fgeo + (size_t)f * 8;
      int o = g.fcell[2 * f + ((s & 1) ? 1 : 0)];
      double sig = (s & 1) ? 1.0 : -1.0;  // +1 if the face normal points out of c
      double fh = 0.0, fb = 0.0;           // flux along the face normal
      if (o == kNbWall) {
        double sg = r[R_SGN];
        double wn = wnorm(vx, vy, fg[3], fg[4], sg * fg[0], sg * fg[1]);
        if (wn > 0.0) {
          double vh, vb, ghx, ghy, gbx, gby;
          recon(g, h, hinf, c, s, kk, vh, ghx, ghy);
          recon(g, b, binf, c, s, kk, vb, gbx, gby);
          FaceEq<C> e;
          e.load(r);
          C Ih, Ib;
          interface_avg<C>(e, g.dim, g.nxi, (C)vx, (C)vy, (C)(vx - fg[3]), (C)(vy - fg[4]), (C)vh, (C)vb,
                           (C)ghx, (C)ghy, (C)gbx, (C)gby, Ih, Ib);
          fh = sg * wn * (double)Ih;
          fb = sg * wn * (double)Ib;
        } else if (wn < 0.0) {
          double cx = vx - r[R_VWX], cy = (g.dim == 2) ? vy - r[R_VWY] : 0.0;
          double Hw = r[R_RHOW] * r[R_HWN] * exp(-r[R_LAMW] * (cx * cx + cy * cy));
          fh = sg * wn * Hw;
          fb = sg * wn * (double)g.nxi * 0.5 / r[R_LAMW] * Hw;
        }
      } else {
        double wn = wnorm(vx, vy, fg[3], fg[4], fg[0], fg[1]);
        if (wn != 0.0) {
          bool upc = (wn > 0.0) == ((s & 1) != 0);  // upwind side is c
          double vh, vb, ghx, ghy, gbx, gby;
          if (upc) {
            recon(g, h, hinf, c, s, kk, vh, ghx, ghy);
            recon(g, b, binf, c, s, kk, vb, gbx, gby);
          } else {
            other_side(g, h, hinf, c, s, o, kk, vh, ghx, ghy);
            other_side(g, b, binf, c, s, o, kk, vb, gbx, gby);
          }
          FaceEq<C> e;
          e.load(r);
          C Ih, Ib;
          interface_avg<C>(e, g.dim, g.nxi, (C)vx, (C)vy, (C)(vx - fg[3]), (C)(vy - fg[4]), (C)vh, (C)vb,
                           (C)ghx, (C)ghy, (C)gbx, (C)gby, Ih, Ib);
          fh = wn * (double)Ih;
          fb = wn * (double)Ib;
        }
      }
      if (!kin) { fh = 0.0; fb = 0.0; }
      if (field) {
        dh -= (C)(sig * fg[2] * fh * ivol);
        db -= (C)(sig * fg[2] * fb * ivol);
      }
      if (own) {
        acc[s][0] += wk * fh;
        acc[s][1] += wk * vx * fh;
        if (g.dim == 2) acc[s][2] += wk * vy * fh;
        acc[s][g.dim + 1] += wk * 0.5 * ((vx * vx + vy * vy) * fh + fb);
      }
    }
    if (kin) {
      Dh[(size_t)c * g.nv + k] = field ? (T)dh : (T)0;
      Db[(size_t)c * g.nv + k] = field ? (T)db : (T)0;
    }
  }
  for (int s = 0; s < 2 * g.dim; ++s) {
    int f = g.cf[4 * c + s];
    if (!owns(g, c, s, f)) continue;
    double v[4];
    for (int m = 0; m < nw; ++m) v[m] = wave_sum(acc[s][m]);
    if (lane == 0) {
      if (F) for (int m = 0; m < nw; ++m) F[(size_t)f * nw + m] = v[m];
      if (wall && g.fcell[2 * f + ((s & 1) ? 1 : 0)] == kNbWall) {
        const double* r = rec + (size_t)f * NREC;
        double* o = wall + (size_t)f * (nw + 1);
        o[0] = r[R_RHOW];
        for (int m = 0; m < nw; ++m) o[1 + m] = r[R_SGN] * v[m];
      }
    }
  }
}

// ------------------------------------------------------------------------
// moments
// ------------------------------------------------------------------------
// plain W and q about the velocity of that W (two passes over the velocities)
template <class T>
__global__ __launch_bounds__(256) void k_moments(Dev g, const T* __restrict__ h, const T* __restrict__ b,
                                                 double* __restrict__ W, double* __restrict__ q) {
  int c = blockIdx.x * 4 + (threadIdx.x >> 6);
  int lane = threadIdx.x & 63;
  if (c >= g.ncell) return;
  double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
  for (int k = lane; k < g.nv; k += 64) {
    double hv = (double)h[(size_t)c * g.nv + k], bv = (double)b[(size_t)c * g.nv + k];
    double vx = g.vx[k], vy = g.vy[k], w = g.wk[k];
    a0 += w * hv;
    a1 += w * vx * hv;
    a2 += w * vy * hv;
    a3 += w * 0.5 * ((vx * vx + vy * vy) * hv + bv);
  }
  a0 = wave_sum(a0); a1 = wave_sum(a1); a2 = wave_sum(a2); a3 = wave_sum(a3);
  double ux = a1 / a0, uy = (g.dim == 2) ? a2 / a0 : 0.0;
  double qx = 0, qy = 0;
  for (int k = lane; k < g.nv; k += 64) {
    double hv = (double)h[(size_t)c * g.nv + k], bv = (double)b[(size_t)c * g.nv + k];
    double cx = g.vx[k] - ux, cy = (g.dim == 2) ? g.vy[k] - uy : 0.0;
    double e = (cx * cx + cy * cy) * hv + bv;
    qx += g.wk[k] * 0.5 * cx * e;
    qy += g.wk[k] * 0.5 * cy * e;
  }
  qx = wave_sum(qx); qy = wave_sum(qy);
  if (lane == 0) {
    double* w = W + (size_t)c * g.nw;
    w[0] = a0; w[1] = a1;
    if (g.dim == 2) { w[2] = a2; w[3] = a3; } else { w[2] = a3; }
    if (q) {
      q[(size_t)c * g.dim] = qx;
      if (g.dim == 2) q[(size_t)c * g.dim + 1] = qy;
    }
  }
}

// heat flux 2q = m3 - 2 P d + |d|^2 m1 - d m2 + 2 d (m1.d) - |d|^2 d m0 of a
// moment record shifted by d = V - s
__device__ inline void heat_from_record(const double* M, double Vx, double Vy, int dim, double& qx,
                                        double& qy) {
  double dx = Vx - M[M_SX], dy = (dim == 2) ? Vy - M[M_SY] : 0.0;
  double dd = dx * dx + dy * dy;
  double m1d = M[M_M1X] * dx + M[M_M1Y] * dy;
  qx = 0.5 * (M[M_M3X] - 2.0 * (M[M_PXX] * dx + M[M_PXY] * dy) + dd * M[M_M1X] - dx * M[M_M2] +
              2.0 * dx * m1d - dd * dx * M[M_M0]);
  qy = 0.5 * (M[M_M3Y] - 2.0 * (M[M_PXY] * dx + M[M_PYY] * dy) + dd * M[M_M1Y] - dy * M[M_M2] +
              2.0 * dy * m1d - dd * dy * M[M_M0]);
  if (dim == 1) qy = 0.0;
}

// Step 7 (W^{s+1} = W' + sum_k V Psi (f - g(W'))) and the moment record of f
// about the shift V' (mode 1); mode 0 only writes the record (shift: V of W);
// mode 2 writes the record and the heat flux about V of W
template <class T>
__global__ __launch_bounds__(256) void k_step7(Dev g, int mode, const T* __restrict__ h,
                                               const T* __restrict__ b, const double* __restrict__ crec,
                                               const double* __restrict__ Wp, double* __restrict__ W,
                                               double* __restrict__ q, double* __restrict__ mrec) {
  int c = blockIdx.x * 4 + (threadIdx.x >> 6);
  int lane = threadIdx.x & 63;
  if (c >= g.ncell || g.type[c] == 0) return;
  double sx, sy, rho = 0, lam = 0, hn = 0;
  if (mode == 1) {
    const double* cr = crec + (size_t)c * NCREC;
    rho = cr[C_RHO]; sx = cr[C_UX]; sy = cr[C_UY]; lam = cr[C_LAM]; hn = cr[C_HN];
  } else {
    double l;
    prim_of(g, W + (size_t)c * g.nw, rho, sx, sy, l);
  }
  double m0 = 0, m1x = 0, m1y = 0, m2 = 0, pxx = 0, pxy = 0, pyy = 0, m3x = 0, m3y = 0;
  double g0 = 0, g1 = 0, g2 = 0, g3 = 0;
  bool step = (mode == 1) && g.type[c] == 1;
  for (int k = lane; k < g.nv; k += 64) {
    double hv = (double)h[(size_t)c * g.nv + k], bv = (double)b[(size_t)c * g.nv + k];
    double vx = g.vx[k], vy = g.vy[k], w = g.wk[k];
    double cx = vx - sx, cy = (g.dim == 2) ? vy - sy : 0.0;
    double c2 = cx * cx + cy * cy;
    double e = c2 * hv + bv;
    m0 += w * hv;
    m1x += w * cx * hv;
    m1y += w * cy * hv;
    m2 += w * e;
    pxx += w * cx * cx * hv;
    pxy += w * cx * cy * hv;
    pyy += w * cy * cy * hv;
    m3x += w * cx * e;
    m3y += w * cy * e;
    if (step) {
      double H = hn * exp(-lam * c2), B = (double)g.nxi * 0.5 / lam * H;
      g0 += w * H;
      g1 += w * vx * H;
      g2 += w * vy * H;
      g3 += w * 0.5 * ((vx * vx + vy * vy) * H + B);
    }
  }
  m0 = wave_sum(m0); m1x = wave_sum(m1x); m1y = wave_sum(m1y); m2 = wave_sum(m2);
  pxx = wave_sum(pxx); pxy = wave_sum(pxy); pyy = wave_sum(pyy);
  m3x = wave_sum(m3x); m3y = wave_sum(m3y);
  if (step) { g0 = wave_sum(g0); g1 = wave_sum(g1); g2 = wave_sum(g2); g3 = wave_sum(g3); }
  if (lane != 0) return;
  double* M = mrec + (size_t)c * NMREC;
  M[M_SX] = sx; M[M_SY] = sy; M[M_M0] = m0; M[M_M1X] = m1x; M[M_M1Y] = m1y; M[M_M2] = m2;
  M[M_PXX] = pxx; M[M_PXY] = pxy; M[M_PYY] = pyy; M[M_M3X] = m3x; M[M_M3Y] = m3y;
  if (mode == 2) {
    q[(size_t)c * g.dim] = 0.5 * m3x;
    if (g.dim == 2) q[(size_t)c * g.dim + 1] = 0.5 * m3y;
  }
  if (!step) return;
  // moments of f in lab velocities
  double fm0 = m0, fm1 = m1x + sx * m0, fm2 = m1y + sy * m0;
  double fmE = 0.5 * (m2 + 2.0 * (sx * m1x + sy * m1y) + (sx * sx + sy * sy) * m0);
  double* w = W + (size_t)c * g.nw;
  const double* wp = Wp + (size_t)c * g.nw;
  double fm[4] = {fm0, fm1, fm2, fmE}, gm[4] = {g0, g1, g2, g3};
  if (g.dim == 1) { fm[2] = fmE; gm[2] = g3; }
  for (int m = 0; m < g.nw; ++m) w[m] = wp[m] + (fm[m] - gm[m]);
  double r2, ux, uy, l2;
  prim_of(g, w, r2, ux, uy, l2);
  double qx, qy;
  heat_from_record(M, ux, uy, g.dim, qx, qy);
  q[(size_t)c * g.dim] = qx;
  if (g.dim == 2) q[(size_t)c * g.dim + 1] = qy;
}

// per-cell equilibrium record from W (or W') and the heat flux (given, or
// from a moment record shifted to the velocity of W)
__global__ void k_cellrec(Dev g, const double* __restrict__ W, const double* __restrict__ q,
                          const double* __restrict__ mrec, double* __restrict__ crec) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= g.ncell || g.type[c] == 0) return;
  double rho, ux, uy, lam;
  prim_of(g, W + (size_t)c * g.nw, rho, ux, uy, lam);
  double qx, qy;
  if (mrec) heat_from_record(mrec + (size_t)c * NMREC, ux, uy, g.dim, qx, qy);
  else { qx = q[(size_t)c * g.dim]; qy = (g.dim == 2) ? q[(size_t)c * g.dim + 1] : 0.0; }
  double* r = crec + (size_t)c * NCREC;
  r[C_RHO] = rho; r[C_UX] = ux; r[C_UY] = uy; r[C_LAM] = lam; r[C_QX] = qx; r[C_QY] = qy;
  r[C_HN] = rho * pow(lam / kPi, 0.5 * g.dim);
  r[C_SH] = 4.0 * (1.0 - g.pr) * lam * lam / (5.0 * rho);
  r[C_ITAU] = inv_tau_of(g, rho, lam);
}

// Shakhov equilibrium h+, b+ of a cell record at velocity (vx, vy)
__device__ inline void cell_fplus(const double* r, int dim, int nxi, double vx, double vy, double& hp,
                                  double& bp) {
  double cx = vx - r[C_UX], cy = (dim == 2) ? vy - r[C_UY] : 0.0;
  double c2 = cx * cx + cy * cy;
  double lam = r[C_LAM];
  double H = r[C_HN] * exp(-lam * c2);
  double rt = 0.5 / lam;
  double B = (double)nxi * rt * H;
  double s = r[C_SH] * (cx * r[C_QX] + cy * r[C_QY]);
  double tl = 2.0 * lam * c2;
  hp = H + s * (tl - 2.0 - dim) * H;
  bp = B + s * (tl - dim) * (double)nxi * rt * H;
}

// Steps 1-2: S = f/dt + (D + (f+ - f)/tau)/2 on field cells
template <class T>
__global__ void k_source(Dev g, double dt, const T* __restrict__ h, const T* __restrict__ b,
                         const double* __restrict__ crec, T* __restrict__ Sh, T* __restrict__ Sb) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t n = (size_t)g.ncell * g.nv;
  if (i >= n) return;
  int c = (int)(i / g.nv), k = (int)(i % g.nv);
  if (g.type[c] != 1) { Sh[i] = (T)0; Sb[i] = (T)0; return; }
  const double* r = crec + (size_t)c * NCREC;
  double hp, bp;
  cell_fplus(r, g.dim, g.nxi, g.vx[k], g.vy[k], hp, bp);
  double hv = (double)h[i], bv = (double)b[i], it = r[C_ITAU];
  // D is passed in Sh/Sb on entry
  double dh = (double)Sh[i], db = (double)Sb[i];
  Sh[i] = (T)(hv / dt + 0.5 * (dh + (hp - hv) * it));
  Sb[i] = (T)(bv / dt + 0.5 * (db + (bp - bv) * it));
}

template <class T>
__global__ void k_maxwellian(Dev g, const double* __restrict__ W, T* __restrict__ h, T* __restrict__ b) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t n = (size_t)g.ncell * g.nv;
  if (i >= n) return;
  int c = (int)(i / g.nv), k = (int)(i % g.nv);
  double rho, ux, uy, lam;
  prim_of(g, W + (size_t)c * g.nw, rho, ux, uy, lam);
  double cx = g.vx[k] - ux, cy = (g.dim == 2) ? g.vy[k] - uy : 0.0;
  double H = rho * pow(lam / kPi, 0.5 * g.dim) * exp(-lam * (cx * cx + cy * cy));
  h[i] = (T)H;
  b[i] = (T)((double)g.nxi * 0.5 / lam * H);
}

// overset interpolation: one wavefront per receptor
template <class T>
__global__ __launch_bounds__(256) void k_interp(Dev g, int nrec, const int* __restrict__ rec,
                                                const int* __restrict__ ptr, const int* __restrict__ don,
                                                const double* __restrict__ wt, T* __restrict__ h,
                                                T* __restrict__ b, double* __restrict__ W,
                                                double* __restrict__ q) {
  int r = blockIdx.x * 4 + (threadIdx.x >> 6);
  int lane = threadIdx.x & 63;
  if (r >= nrec) return;
  int c = rec[r], p0 = ptr[r], p1 = ptr[r + 1];
  for (int k = lane; k < g.nv; k += 64) {
    double sh = 0, sb = 0;
    for (int p = p0; p < p1; ++p) {
      sh += wt[p] * (double)h[(size_t)don[p] * g.nv + k];
      sb += wt[p] * (double)b[(size_t)don[p] * g.nv + k];
    }
    h[(size_t)c * g.nv + k] = (T)sh;
    b[(size_t)c * g.nv + k] = (T)sb;
  }
  if (lane < g.nw) {
    double s = 0;
    for (int p = p0; p < p1; ++p) s += wt[p] * W[(size_t)don[p] * g.nw + lane];
    W[(size_t)c * g.nw + lane] = s;
  }
  if (q && lane >= 8 && lane < 8 + g.dim) {
    int m = lane - 8;
    double s = 0;
    for (int p = p0; p < p1; ++p) s += wt[p] * q[(size_t)don[p] * g.dim + m];
    q[(size_t)c * g.dim + m] = s;
  }
}

// ------------------------------------------------------------------------
// macro LU-SGS (Eq. dualTimeStepping_macro)
// ------------------------------------------------------------------------
// spectral radius per face from W^s
__global__ void k_gamma(Dev g, const double* __restrict__ W, double* __restrict__ gam) {
  int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= g.nface) return;
  int L = g.fcell[2 * f], R = g.fcell[2 * f + 1];
  const double* fg = g.fgeo + (size_t)f * 8;
  double gma = (double)(g.dim + g.nxi + 2) / (double)(g.dim + g.nxi);
  auto state = [&](int code, int other, double& ux, double& uy, double& a) {
    const double* w;
    if (code >= 0) w = W + (size_t)code * g.nw;
    else if (code == kNbFar) w = g.winf;
    else w = W + (size_t)other * g.nw;
    double rho, lam;
    prim_of(g, w, rho, ux, uy, lam);
    a = sqrt(gma * 0.5 / lam);
  };
  if (L == kNbWall || R == kNbWall) {
    int c = (L == kNbWall) ? R : L;
    if (c < 0) { gam[f] = 0.0; return; }
    double ux, uy, a;
    state(c, c, ux, uy, a);
    gam[f] = fabs((ux - fg[3]) * fg[0] + (uy - fg[4]) * fg[1]) + a;
    return;
  }
  int inner = (L >= 0) ? L : R;
  if (inner < 0) { gam[f] = 0.0; return; }
  double u1, v1, a1, u2, v2, a2;
  state(L, inner, u1, v1, a1);
  state(R, inner, u2, v2, a2);
  double mx = 0.5 * (u1 + u2), my = 0.5 * (v1 + v2);
  gam[f] = fabs((mx - fg[3]) * fg[0] + (my - fg[4]) * fg[1]) + 0.5 * (a1 + a2);
}

// residual R and LU-SGS diagonal per field cell
__global__ void k_macro_prep(Dev g, double dt, const double* __restrict__ W, const double* __restrict__ Wn,
                             const double* __restrict__ F, const double* __restrict__ Fn,
                             const double* __restrict__ gam, double* __restrict__ R,
                             double* __restrict__ Dg) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= g.ncell) return;
  int nw = g.nw;
  if (g.type[c] != 1) {
    for (int m = 0; m < nw; ++m) R[(size_t)c * nw + m] = 0.0;
    Dg[c] = 1.0;
    return;
  }
  double ivol = 1.0 / g.vol[c];
  double r[4], sg = 0.0;
  for (int m = 0; m < nw; ++m) r[m] = -(W[(size_t)c * nw + m] - Wn[(size_t)c * nw + m]) / dt;
  for (int s = 0; s < 2 * g.dim; ++s) {
    int f = g.cf[4 * c + s];
    if (f < 0) continue;
    double S = g.fgeo[(size_t)f * 8 + 2];
    double sig = (s & 1) ? 1.0 : -1.0;
    for (int m = 0; m < nw; ++m)
      r[m] -= 0.5 * ivol * sig * S * (F[(size_t)f * nw + m] + Fn[(size_t)f * nw + m]);
    sg += S * gam[f];
  }
  for (int m = 0; m < nw; ++m) R[(size_t)c * nw + m] = r[m];
  Dg[c] = 1.0 / g.dtp[c] + 1.0 / dt + 0.25 * ivol * sg;
}

// ALE Euler flux difference F_E(W + dW) - F_E(W) along n with mesh velocity U
__device__ inline void euler_dflux(int dim, int nxi, const double* W, const double* dW, double nx, double ny,
                                   double ux, double uy, double* out) {
  auto fe = [&](const double* w, double* o) {
    double rho = w[0], vx = w[1] / rho, vy = (dim == 2) ? w[2] / rho : 0.0;
    double e = w[dim + 1] - 0.5 * rho * (vx * vx + vy * vy);
    double p = 2.0 * e / (double)(dim + nxi);  // rho/(2 lam)
    double th = (vx - ux) * nx + ((dim == 2) ? (vy - uy) * ny : 0.0);
    o[0] = rho * th;
    o[1] = w[1] * th + p * nx;
    if (dim == 2) o[2] = w[2] * th + p * ny;
    o[dim + 1] = w[dim + 1] * th + p * (vx * nx + ((dim == 2) ? vy * ny : 0.0));
  };
  double w1[4], f1[4], f0[4];
  for (int m = 0; m < dim + 2; ++m) w1[m] = W[m] + dW[m];
  fe(w1, f1);
  fe(W, f0);
  for (int m = 0; m < dim + 2; ++m) out[m] = f1[m] - f0[m];
}

// ------------------------------------------------------------------------
// hyperplane LU-SGS sweeps
//
// Within a block the cells are ordered lexicographically (i fastest).  The
// lower neighbours of (i, j) are (i-1, j), (i, j-1) and, across a periodic
// seam, (0, j) for i = ni-1 and (i, 0) for j = nj-1; all of them lie on an
// earlier hyperplane i + j, so sweeping hyperplanes in order reproduces the
// sequential Gauss-Seidel order exactly.  Each thread owns `rpt` contiguous
// rows and keeps the latest value of each row in registers; the first row of
// a thread reads the last row of the previous thread through LDS.
// ------------------------------------------------------------------------
constexpr int kMaxRowsMacro = 8;
constexpr int kMaxRowsMicro = 4;

__device__ inline void macro_couple(const Dev& g, const double* __restrict__ W,
                                    const double* __restrict__ gam, int c, int s, int nbc,
                                    const double* x, double* acc) {
  if (g.type[nbc] != 1) return;
  int f = g.cf[4 * c + s];
  const double* fg = g.fgeo + (size_t)f * 8;
  double sg = (s & 1) ? 1.0 : -1.0;
  double dF[4];
  euler_dflux(g.dim, g.nxi, W + (size_t)nbc * g.nw, x, sg * fg[0], sg * fg[1], fg[3], fg[4], dF);
  double G = gam[f], S = fg[2];
  for (int m = 0; m < g.nw; ++m) acc[m] += S * (dF[m] - G * x[m]);
}

__global__ __launch_bounds__(64) void k_macro_sweep(Dev g, const int* __restrict__ binfo,
                                                    const double* __restrict__ W,
                                                    const double* __restrict__ R,
                                                    const double* __restrict__ Dg,
                                                    const double* __restrict__ gam,
                                                    double* __restrict__ dWs, double* __restrict__ dW,
                                                    double* __restrict__ Wp, double* __restrict__ rpart) {
  const int* bi = binfo + 8 * blockIdx.x;
  const int ni = bi[0], nj = bi[1], c0 = bi[2], pi = bi[3], pj = bi[4];
  const int t = threadIdx.x, NT = blockDim.x;
  const int rpt = (nj + NT - 1) / NT;
  const int j0 = t * rpt;
  const int nw = g.nw;
  __shared__ double hand[2][64][4];
  __shared__ double pjb[64][4];
  double prev[kMaxRowsMacro][4], cw[kMaxRowsMacro][4];
  for (int r = 0; r < kMaxRowsMacro; ++r)
    for (int m = 0; m < 4; ++m) { prev[r][m] = 0.0; cw[r][m] = 0.0; }
  // residual norm over the block's field cells
  double rs[4] = {0, 0, 0, 0};
  for (int r = 0; r < rpt; ++r) {
    int j = j0 + r;
    if (j >= nj) break;
    for (int i = 0; i < ni; ++i) {
      int c = c0 + i + ni * j;
      if (g.type[c] != 1) continue;
      for (int m = 0; m < nw; ++m) rs[m] += R[(size_t)c * nw + m] * R[(size_t)c * nw + m];
    }
  }
  for (int m = 0; m < 4; ++m) rs[m] = wave_sum(rs[m]);
  if (t == 0) for (int m = 0; m < nw; ++m) rpart[(size_t)blockIdx.x * 4 + m] = rs[m];
  const int H = ni + nj - 1;
  // forward sweep: (D + L) dW* = R
  for (int h = 0; h < H; ++h) {
    for (int r = rpt - 1; r >= 0; --r) {
      int j = j0 + r, i = h - j;
      if (j >= nj || i < 0 || i >= ni) continue;
      int c = c0 + i + ni * j;
      double x[4] = {0, 0, 0, 0};
      if (g.type[c] == 1) {
        double acc[4] = {0, 0, 0, 0};
        if (i >= 1) macro_couple(g, W, gam, c, 0, c - 1, prev[r], acc);
        if (j >= 1) macro_couple(g, W, gam, c, 2, c - ni, (r > 0) ? prev[r - 1] : hand[(h - 1) & 1][t - 1], acc);
        if (pi && i == ni - 1 && ni > 1) macro_couple(g, W, gam, c, 1, c - (ni - 1), cw[r], acc);
        if (pj && j == nj - 1 && nj > 1) macro_couple(g, W, gam, c, 3, c0 + i, pjb[i], acc);
        double ivd = 0.25 / g.vol[c];
        for (int m = 0; m < nw; ++m) x[m] = (R[(size_t)c * nw + m] - ivd * acc[m]) / Dg[c];
      }
      for (int m = 0; m < nw; ++m) {
        dWs[(size_t)c * nw + m] = x[m];
        prev[r][m] = x[m];
        if (i == 0) cw[r][m] = x[m];
        if (r == rpt - 1) hand[h & 1][t][m] = x[m];
        if (pj && j == 0) pjb[i][m] = x[m];
      }
    }
    __syncthreads();
  }
  for (int r = 0; r < kMaxRowsMacro; ++r)
    for (int m = 0; m < 4; ++m) { prev[r][m] = 0.0; cw[r][m] = 0.0; }
  __syncthreads();
  // backward sweep: (D + U) dW = D dW*
  for (int h = H - 1; h >= 0; --h) {
    for (int r = 0; r < rpt; ++r) {
      int j = j0 + r, i = h - j;
      if (j >= nj || i < 0 || i >= ni) continue;
      int c = c0 + i + ni * j;
      double x[4] = {0, 0, 0, 0};
      if (g.type[c] == 1) {
        double acc[4] = {0, 0, 0, 0};
        if (i + 1 < ni) macro_couple(g, W, gam, c, 1, c + 1, prev[r], acc);
        if (j + 1 < nj) macro_couple(g, W, gam, c, 3, c + ni, (r + 1 < rpt) ? prev[r + 1] : hand[(h + 1) & 1][t + 1], acc);
        if (pi && i == 0 && ni > 1) macro_couple(g, W, gam, c, 0, c + ni - 1, cw[r], acc);
        if (pj && j == 0 && nj > 1) macro_couple(g, W, gam, c, 2, c0 + i + ni * (nj - 1), pjb[i], acc);
        double ivd = 0.25 / (g.vol[c] * Dg[c]);
        for (int m = 0; m < nw; ++m) x[m] = dWs[(size_t)c * nw + m] - ivd * acc[m];
      }
      for (int m = 0; m < nw; ++m) {
        dW[(size_t)c * nw + m] = x[m];
        Wp[(size_t)c * nw + m] = W[(size_t)c * nw + m] + x[m];
        prev[r][m] = x[m];
        if (i == ni - 1) cw[r][m] = x[m];
        if (r == 0) hand[h & 1][t][m] = x[m];
        if (pj && j == nj - 1) pjb[i][m] = x[m];
      }
    }
    __syncthreads();
  }
}

// L2 norms of the residual: sum the per-block partial sums
__global__ void k_resid(int nblock, int nw, const double* __restrict__ rpart, double* __restrict__ out) {
  int m = threadIdx.x;
  if (m >= nw) return;
  double s = 0.0;
  for (int b = 0; b < nblock; ++b) s += rpart[(size_t)b * 4 + m];
  out[m] = sqrt(s);
}

// micro LU-SGS (Eq. dualTimeStepping_micro), forward and backward sweep of
// one velocity chunk of one block; Dh/Db hold the flux divergence on entry
// and dF* afterwards; h, b are updated to f^{s+1}
template <class T>
__global__ __launch_bounds__(1024) void k_micro(Dev g, const int* __restrict__ binfo, int KC, double dt,
                                                const double* __restrict__ crec, T* __restrict__ h,
                                                T* __restrict__ b, const T* __restrict__ Sh,
                                                const T* __restrict__ Sb, T* __restrict__ Dh,
                                                T* __restrict__ Db) {
  extern __shared__ double smem[];
  const int* bi = binfo + 8 * blockIdx.y;
  const int ni = bi[0], nj = bi[1], c0 = bi[2], pi = bi[3], pj = bi[4];
  const int t = threadIdx.x, nslot = blockDim.x / KC;
  const int lk = t % KC, slot = t / KC;
  const int k = blockIdx.x * KC + lk;
  const bool kin = k < g.nv;
  const int kk = kin ? k : g.nv - 1;
  const int rpt = (nj + nslot - 1) / nslot;
  const int j0 = slot * rpt;
  // LDS: hand[2][nslot][KC][2], then pj[ni][KC][2]
  double* hand = smem;
  double* pjb = smem + 2 * nslot * KC * 2;
  auto H_ = [&](int p, int s) -> double* { return hand + ((size_t)(p * nslot + s) * KC + lk) * 2; };
  auto P_ = [&](int i) -> double* { return pjb + ((size_t)i * KC + lk) * 2; };
  const double vx = g.vx[kk], vy = g.vy[kk];
  double ph[kMaxRowsMicro], pb[kMaxRowsMicro], ch[kMaxRowsMicro], cb[kMaxRowsMicro];
  for (int r = 0; r < kMaxRowsMicro; ++r) { ph[r] = pb[r] = ch[r] = cb[r] = 0.0; }
  const int HH = ni + nj - 1;
  const double idt = 1.0 / dt;

  auto diag_and_w = [&](int c, double* wn, double& d) {
    const double* cr = crec + (size_t)c * NCREC;
    double ivol = 1.0 / g.vol[c];
    d = 1.0 / g.dtp[c] + idt + 0.5 * cr[C_ITAU];
    for (int s = 0; s < 2 * g.dim; ++s) {
      int f = g.cf[4 * c + s];
      wn[s] = 0.0;
      if (f < 0) continue;
      const double* fg = g.fgeo + (size_t)f * 8;
      double w = wnorm(vx, vy, fg[3], fg[4], fg[0], fg[1]);
      w = (s & 1) ? w : -w;
      wn[s] = w;
      d += 0.5 * ivol * fg[2] * ((w > 0.0) ? w : 0.0);
    }
  };
  // forward sweep
  for (int hp = 0; hp < HH; ++hp) {
    for (int r = rpt - 1; r >= 0; --r) {
      int j = j0 + r, i = hp - j;
      if (j >= nj || i < 0 || i >= ni) continue;
      int c = c0 + i + ni * j;
      double xh = 0.0, xb = 0.0;
      if (g.type[c] == 1) {
        double wn[4], d;
        diag_and_w(c, wn, d);
        double oh = 0.0, ob = 0.0;
        auto couple = [&](int s, double vh, double vb) {
          int f = g.cf[4 * c + s];
          double S = g.fgeo[(size_t)f * 8 + 2];
          double wm = (wn[s] < 0.0) ? wn[s] : 0.0;
          oh += S * wm * vh;
          ob += S * wm * vb;
        };
        if (i >= 1) couple(0, ph[r], pb[r]);
        if (j >= 1) {
          if (r > 0) couple(2, ph[r - 1], pb[r - 1]);
          else { double* q = H_((hp - 1) & 1, slot - 1); couple(2, q[0], q[1]); }
        }
        if (pi && i == ni - 1 && ni > 1) couple(1, ch[r], cb[r]);
        if (pj && j == nj - 1 && nj > 1) { double* q = P_(i); couple(3, q[0], q[1]); }
        const double* cr = crec + (size_t)c * NCREC;
        double hpl, bpl;
        cell_fplus(cr, g.dim, g.nxi, vx, vy, hpl, bpl);
        size_t o = (size_t)c * g.nv + kk;
        double hv = (double)h[o], bv = (double)b[o];
        double it = cr[C_ITAU];
        double rh = (double)Sh[o] - hv * idt + 0.5 * ((double)Dh[o] + (hpl - hv) * it);
        double rb = (double)Sb[o] - bv * idt + 0.5 * ((double)Db[o] + (bpl - bv) * it);
        double ivol2 = 0.5 / g.vol[c];
        xh = (rh - ivol2 * oh) / d;
        xb = (rb - ivol2 * ob) / d;
        if (kin) { Dh[o] = (T)xh; Db[o] = (T)xb; }
      }
      ph[r] = xh; pb[r] = xb;
      if (i == 0) { ch[r] = xh; cb[r] = xb; }
      if (r == rpt - 1) { double* q = H_(hp & 1, slot); q[0] = xh; q[1] = xb; }
      if (pj && j == 0) { double* q = P_(i); q[0] = xh; q[1] = xb; }
    }
    __syncthreads();
  }
  for (int r = 0; r < kMaxRowsMicro; ++r) { ph[r] = pb[r] = ch[r] = cb[r] = 0.0; }
  __syncthreads();
  // backward sweep
  for (int hp = HH - 1; hp >= 0; --hp) {
    for (int r = 0; r < rpt; ++r) {
      int j = j0 + r, i = hp - j;
      if (j >= nj || i < 0 || i >= ni) continue;
      int c = c0 + i + ni * j;
      double xh = 0.0, xb = 0.0;
      if (g.type[c] == 1) {
        double wn[4], d;
        diag_and_w(c, wn, d);
        double oh = 0.0, ob = 0.0;
        auto couple = [&](int s, double vh, double vb) {
          int f = g.cf[4 * c + s];
          double S = g.fgeo[(size_t)f * 8 + 2];
          double wm = (wn[s] < 0.0) ? wn[s] : 0.0;
          oh += S * wm * vh;
          ob += S * wm * vb;
        };
        if (i + 1 < ni) couple(1, ph[r], pb[r]);
        if (j + 1 < nj) {
          if (r + 1 < rpt) couple(3, ph[r + 1], pb[r + 1]);
          else { double* q = H_((hp + 1) & 1, slot + 1); couple(3, q[0], q[1]); }
        }
        if (pi && i == 0 && ni > 1) couple(0, ch[r], cb[r]);
        if (pj && j == 0 && nj > 1) { double* q = P_(i); couple(2, q[0], q[1]); }
        size_t o = (size_t)c * g.nv + kk;
        double ivd = 0.5 / (g.vol[c] * d);
        xh = (double)Dh[o] - ivd * oh;
        xb = (double)Db[o] - ivd * ob;
        if (kin) {
          h[o] = (T)((double)h[o] + xh);
          b[o] = (T)((double)b[o] + xb);
        }
      }
      ph[r] = xh; pb[r] = xb;
      if (i == ni - 1) { ch[r] = xh; cb[r] = xb; }
      if (r == 0) { double* q = H_(hp & 1, slot); q[0] = xh; q[1] = xb; }
      if (pj && j == nj - 1) { double* q = P_(i); q[0] = xh; q[1] = xb; }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------------
// host launchers
// ------------------------------------------------------------------------
static inline unsigned nb4(int n) { return (unsigned)((n + 3) / 4); }
static inline unsigned nbl(size_t n, int t) { return (unsigned)((n + t - 1) / t); }

template <class T, class C>
void launch_flux_t(const Dev& g, double dts, const void* h, const void* b, const double* W, const double* q,
                   double* gW, double* rec, void* Dh, void* Db, double* F, double* wall, hipStream_t st,
                   hipEvent_t* ev) {
  k_gradW<<<nbl(g.ncell, 256), 256, 0, st>>>(g, W, gW);
  k_wallprep<<<nbl(g.nface, 256), 256, 0, st>>>(g, dts, W, q, gW, rec);
  if (ev) (void)hipEventRecord(ev[0], st);
  k_face_eq<T><<<nb4(g.ncell), 256, 0, st>>>(g, dts, (const T*)h, (const T*)b, W, gW, rec);
  if (ev) (void)hipEventRecord(ev[1], st);
  k_flux<T, C><<<nb4(g.ncell), 256, 0, st>>>(g, (const T*)h, (const T*)b, rec, (T*)Dh, (T*)Db, F, wall);
}

void launch_flux(const Dev& g, int prec, double dts, const void* h, const void* b, const double* W,
                 const double* q, double* gW, double* rec, void* Dh, void* Db, double* F, double* wall,
                 hipStream_t st, hipEvent_t* ev) {
  if (prec == 0) launch_flux_t<double, double>(g, dts, h, b, W, q, gW, rec, Dh, Db, F, wall, st, ev);
  else launch_flux_t<float, float>(g, dts, h, b, W, q, gW, rec, Dh, Db, F, wall, st, ev);
}

void launch_moments(const Dev& g, int prec, const void* h, const void* b, double* W, double* q, hipStream_t st) {
  if (prec == 0) k_moments<double><<<nb4(g.ncell), 256, 0, st>>>(g, (const double*)h, (const double*)b, W, q);
  else k_moments<float><<<nb4(g.ncell), 256, 0, st>>>(g, (const float*)h, (const float*)b, W, q);
}

void launch_maxwellian(const Dev& g, int prec, const double* W, void* h, void* b, hipStream_t st) {
  size_t n = (size_t)g.ncell * g.nv;
  if (prec == 0) k_maxwellian<double><<<nbl(n, 256), 256, 0, st>>>(g, W, (double*)h, (double*)b);
  else k_maxwellian<float><<<nbl(n, 256), 256, 0, st>>>(g, W, (float*)h, (float*)b);
}

void launch_interp(const Dev& g, int prec, int nrec, const int* rec, const int* ptr, const int* don,
                   const double* w, void* h, void* b, double* W, double* q, hipStream_t st) {
  if (nrec <= 0) return;
  if (prec == 0) k_interp<double><<<nb4(nrec), 256, 0, st>>>(g, nrec, rec, ptr, don, w, (double*)h, (double*)b, W, q);
  else k_interp<float><<<nb4(nrec), 256, 0, st>>>(g, nrec, rec, ptr, don, w, (float*)h, (float*)b, W, q);
}

void launch_cellrec(const Dev& g, const double* W, const double* q, const double* mrec, double* crec,
                    hipStream_t st) {
  k_cellrec<<<nbl(g.ncell, 256), 256, 0, st>>>(g, W, q, mrec, crec);
}

void launch_source(const Dev& g, int prec, double dt, const void* h, const void* b, const double* crec,
                   void* Sh, void* Sb, hipStream_t st) {
  size_t n = (size_t)g.ncell * g.nv;
  if (prec == 0) k_source<double><<<nbl(n, 256), 256, 0, st>>>(g, dt, (const double*)h, (const double*)b, crec, (double*)Sh, (double*)Sb);
  else k_source<float><<<nbl(n, 256), 256, 0, st>>>(g, dt, (const float*)h, (const float*)b, crec, (float*)Sh, (float*)Sb);
}

void launch_step7(const Dev& g, int prec, int mode, const void* h, const void* b, const double* crec,
                  const double* Wp, double* W, double* q, double* mrec, hipStream_t st) {
  if (prec == 0) k_step7<double><<<nb4(g.ncell), 256, 0, st>>>(g, mode, (const double*)h, (const double*)b, crec, Wp, W, q, mrec);
  else k_step7<float><<<nb4(g.ncell), 256, 0, st>>>(g, mode, (const float*)h, (const float*)b, crec, Wp, W, q, mrec);
}

void launch_macro(const Dev& g, const int* binfo, double dt, const double* W, const double* Wn,
                  const double* F, const double* Fn, double* gam, double* R, double* Dg, double* dWs,
                  double* dW, double* Wp, double* rpart, double* resid, hipStream_t st) {
  k_gamma<<<nbl(g.nface, 256), 256, 0, st>>>(g, W, gam);
  k_macro_prep<<<nbl(g.ncell, 256), 256, 0, st>>>(g, dt, W, Wn, F, Fn, gam, R, Dg);
  k_macro_sweep<<<g.nblock, 64, 0, st>>>(g, binfo, W, R, Dg, gam, dWs, dW, Wp, rpart);
  if (resid) k_resid<<<1, 64, 0, st>>>(g.nblock, g.nw, rpart, resid);
}

void launch_micro(const Dev& g, int prec, const int* binfo, int max_ni, int max_nj, int any_pj, double dt,
                  const double* crec, void* h, void* b, const void* Sh, const void* Sb, void* Dh, void* Db,
                  hipStream_t st) {
  int KC, nslot;
  if (g.dim == 1) { KC = 64; nslot = 1; }
  else {
    KC = 16;
    nslot = max_nj < 64 ? ((max_nj + 3) / 4) * 4 : 64;
  }
  size_t lds = sizeof(double) * (size_t)(2 * nslot * KC * 2 + (any_pj ? max_ni * KC * 2 : 0));
  dim3 grid((unsigned)((g.nv + KC - 1) / KC), (unsigned)g.nblock);
  if (prec == 0)
    k_micro<double><<<grid, nslot * KC, lds, st>>>(g, binfo, KC, dt, crec, (double*)h, (double*)b,
                                                   (const double*)Sh, (const double*)Sb, (double*)Dh, (double*)Db);
  else
    k_micro<float><<<grid, nslot * KC, lds, st>>>(g, binfo, KC, dt, crec, (float*)h, (float*)b,
                                                  (const float*)Sh, (const float*)Sb, (float*)Dh, (float*)Db);
}

}  // namespace ugks
