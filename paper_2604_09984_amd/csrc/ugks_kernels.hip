// HIP kernels (gfx950, wave64) of one dual-time pseudo-iteration of the
// implicit unsteady UGKS on moving overset structured meshes.
//
// Layout: h, b [ncell][nv] velocity innermost, so a wavefront whose lanes are
// 64 consecutive velocities reads 64 consecutive values of one cell.
// Velocity reductions are wavefront shuffles accumulated in double.
#include "ugks_kernels.h"

#include <mutex>
#include <vector>

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

// interface distribution integrated over dt_s and divided by dt_s
// (Eq. fullSolution with the coefficient integrals) for h (m = 0) and b
// (m = 1), computed in type C
template <class C>
struct FaceEq {
  C ux, uy, lam, rt, sqx, sqy, hn, ax[4], ay[4], at[4], t[5];
  __device__ void load(const double* r) {
    ux = (C)r[R_UX]; uy = (C)r[R_UY]; lam = (C)r[R_LAM]; rt = (C)r[R_RT];
    sqx = (C)r[R_SQX]; sqy = (C)r[R_SQY]; hn = (C)r[R_HN];
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
  const C rt = e.rt;
  C B = C(nxi) * rt * H;
  C s = cx * e.sqx + cy * e.sqy;
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

// read-only tables of a launch (face records, packed face geometry, block
// table) addressed in the constant address space: wave-uniform entries are
// scalar loads wherever the table pointer comes from (a kernel argument or
// the case table of a batched launch)
typedef const double __attribute__((address_space(4))) cdouble;
typedef const int __attribute__((address_space(4))) cint;

// 2D form of interface_avg from the per-face polynomials of the record
// (record_derived): c = v - U, w = v - Uf
template <class C, class RP>
__device__ __forceinline__ void interface_poly(RP r, C cx, C cy, C wx, C wy, C fh, C fb, C ghx, C ghy,
                                               C gbx, C gby, C& Ih, C& Ib) {
  const C E = expo<C>(-(C)r[R_LAM] * (cx * cx + cy * cy));
  const auto p = r + R_PH;
  const C p0 = (C)p[0] + cy * ((C)p[1] + cy * ((C)p[2] + cy * (C)p[3]));
  const C p1 = (C)p[4] + cy * ((C)p[5] + cy * (C)p[6]);
  const C p2 = (C)p[7] + cy * (C)p[8];
  const C Qh = p0 + cx * (p1 + cx * (p2 + cx * (C)p[9]));
  const C Qb = (C)r[R_KB] * Qh + ((C)r[R_LB] + cx * (C)r[R_LB + 1] + cy * (C)r[R_LB + 2]);
  const C t0 = (C)r[R_T1], t1 = (C)r[R_T1 + 1];
  Ih = t0 * fh + t1 * (wx * ghx + wy * ghy) + E * Qh;
  Ib = t0 * fb + t1 * (wx * gbx + wy * gby) + E * Qb;
}

// ------------------------------------------------------------------------
// cell gradients of W (limited, physical): gW[cell][2][nw]
// ------------------------------------------------------------------------
__device__ __forceinline__ void gradW_body(int BX, const Dev& g, const double* __restrict__ W, double* __restrict__ gW) {
  int c = BX * blockDim.x + threadIdx.x;
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
__global__ void k_gradW(Dev g, const double* __restrict__ W, double* __restrict__ gW) {
  gradW_body(blockIdx.x, g, W, gW);
}

// ------------------------------------------------------------------------
// wall incident state of every active wall face (one-sided data of the
// interior cell): record fields R_RHO..R_T1, wall parameters, sign
// ------------------------------------------------------------------------
__device__ __forceinline__ void wallprep_body(int BX, const Dev& g, double dts, const double* __restrict__ W,
                                              const double* __restrict__ q, const double* __restrict__ gW,
                                              double* __restrict__ rec) {
  int f = BX * blockDim.x + threadIdx.x;
  if (f >= g.nface) return;
  int L = g.fcell[2 * f], R = g.fcell[2 * f + 1];
  double* r = rec + (size_t)f * NREC;
  if (L != kNbWall && R != kNbWall) {
    // moment shift: mean velocity of the two sides (a ghost side is the far
    // field or a copy of the interior cell)
    const int inner = (L >= 0) ? L : R;
    if (inner < 0) return;
    auto vel = [&](int code, double& ax, double& ay) {
      const double* Wc = (code >= 0) ? W + (size_t)code * g.nw
                                     : ((code == kNbFar) ? g.winf : W + (size_t)inner * g.nw);
      ax = Wc[1] / Wc[0];
      ay = (g.dim == 2) ? Wc[2] / Wc[0] : 0.0;
    };
    double u1, v1, u2, v2;
    vel(L, u1, v1);
    vel(R, u2, v2);
    r[R_SX] = 0.5 * (u1 + u2);
    r[R_SY] = 0.5 * (v1 + v2);
    return;
  }
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
  // a non-physical extrapolation falls back to the cell state
  if (!physical_state(g.dim, Win))
    for (int m = 0; m < nw; ++m) Win[m] = W[(size_t)c * nw + m];
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
  record_derived(r, g.dim, g.nxi, fg[3], fg[4]);
  r[R_LAMW] = 0.5 / fg[7];
  r[R_HWN] = pow(r[R_LAMW] / kPi, 0.5 * g.dim);
  r[R_VWX] = fg[5];
  r[R_VWY] = fg[6];
  r[R_SGN] = (R == kNbWall) ? 1.0 : -1.0;
}
__global__ void k_wallprep(Dev g, double dts, const double* __restrict__ W, const double* __restrict__ q,
                           const double* __restrict__ gW, double* __restrict__ rec) {
  wallprep_body(blockIdx.x, g, dts, W, q, gW, rec);
}

// ------------------------------------------------------------------------
// face equilibrium and flux: one wavefront per cell, lanes over velocities.
// The cell index is wave-uniform, so topology, geometry and face records
// come through scalar loads; each neighbour value is loaded once per
// velocity and shared by the cell's own reconstruction and the neighbours'.
// ------------------------------------------------------------------------
__device__ __forceinline__ double exact_wn(double vx, double vy, double ux, double uy, double nx, double ny) {
#pragma clang fp contract(off)
  double a = (vx - ux) * nx;
  double b = (vy - uy) * ny;
  return a + b;
}

__device__ __forceinline__ double lim(int lo, int hi, double vlo, double v0, double vhi) {
  if (lo == kNbMiss || hi == kNbMiss) return 0.0;
  if (lo == kNbWall && hi == kNbWall) return 0.0;
  if (lo == kNbWall) return vhi - v0;
  if (hi == kNbWall) return v0 - vlo;
  double s1 = v0 - vlo, s2 = vhi - v0;
  double vl = (s1 * fabs(s2) + fabs(s1) * s2) / (fabs(s1) + fabs(s2));
  return (s1 * s2 <= 0.0) ? 0.0 : vl;
}

template <class T>
__device__ __forceinline__ double fetch(const T* __restrict__ f, const T* __restrict__ finf, int code, double self,
                                        int nv, int k) {
  if (code >= 0) return (double)f[(size_t)code * nv + k];
  if (code == kNbFar) return (double)finf[k];
  return self;
}

__device__ __forceinline__ bool owns(const Dev& g, int c, int s, int f) {
  if (f < 0 || !g.fact[f]) return false;
  int other = g.fcell[2 * f + ((s & 1) ? 1 : 0)];
  return (s & 1) || other < 0;
}

// per-velocity data of one distribution component at a cell and its
// neighbours: own value, neighbour values and own physical gradient
template <int D>
struct Local {
  double v0, nbv[2 * D], gx, gy;
};

template <int D, class T>
__device__ __forceinline__ void local_data(const Dev& g, const T* __restrict__ f, const T* __restrict__ finf,
                                           int c, const int* nbc, const double* G, int k, Local<D>& L) {
  L.v0 = (double)f[(size_t)c * g.nv + k];
#pragma unroll
  for (int s = 0; s < 2 * D; ++s) L.nbv[s] = fetch(f, finf, nbc[s], L.v0, g.nv, k);
  double si = lim(nbc[0], nbc[1], L.nbv[0], L.v0, L.nbv[1]);
  double sj = (D == 2) ? lim(nbc[2], nbc[3], L.nbv[2], L.v0, L.nbv[3]) : 0.0;
  L.gx = G[0] * si + G[1] * sj;
  L.gy = (D == 2) ? G[2] * si + G[3] * sj : 0.0;
}

// reconstruction of the neighbour o across slot s of cell c (o's own slot is
// s ^ 1; its neighbour across that face is c with value vc)
template <int D, class T>
__device__ __forceinline__ void neighbour_recon(const Dev& g, const T* __restrict__ f, const T* __restrict__ finf,
                                                int o, int s, double vo, double vc, int k, double& val,
                                                double& gx, double& gy) {
  const int dir = s >> 1;
  const int* nbo = g.nb + 4 * o;
  int lo = nbo[2 * dir], hi = nbo[2 * dir + 1];
  double vlo, vhi;
  if (s & 1) { vlo = vc; vhi = fetch(f, finf, hi, vo, g.nv, k); }  // o on the high side of c
  else { vhi = vc; vlo = fetch(f, finf, lo, vo, g.nv, k); }
  double sd = lim(lo, hi, vlo, vo, vhi);
  double st = 0.0;
  if (D == 2) {
    int t = 1 - dir;
    int tl = nbo[2 * t], th = nbo[2 * t + 1];
    st = lim(tl, th, fetch(f, finf, tl, vo, g.nv, k), vo, fetch(f, finf, th, vo, g.nv, k));
  }
  double si = (dir == 0) ? sd : st, sj = (dir == 0) ? st : sd;
  const double* G = g.G + 4 * o;
  gx = G[0] * si + G[1] * sj;
  gy = (D == 2) ? G[2] * si + G[3] * sj : 0.0;
  const double* cd = g.cdx + 8 * o + 2 * (s ^ 1);
  val = vo + gx * cd[0] + gy * cd[1];
}

template <int D, class T>
__global__ __launch_bounds__(256) void k_face_eq(Dev g, double dts, const T* __restrict__ h,
                                                 const T* __restrict__ b, const double* __restrict__ W,
                                                 const double* __restrict__ gW, double* __restrict__ rec) {
  const int c = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
  const int lane = threadIdx.x & 63;
  if (c >= g.ncell || g.type[c] == 0) return;
  const T* hinf = (const T*)g.finf_h;
  const T* binf = (const T*)g.finf_b;
  const int nw = D + 2;
  int nbc[2 * D];
#pragma unroll
  for (int s = 0; s < 2 * D; ++s) nbc[s] = g.nb[4 * c + s];
  const double* G = g.G + 4 * c;
#pragma unroll
  for (int s = 0; s < 2 * D; ++s) {
    const int f = g.cf[4 * c + s];
    if (!owns(g, c, s, f)) continue;
    const int o = g.fcell[2 * f + ((s & 1) ? 1 : 0)];
    const double* fg = g.fgeo + (size_t)f * 8;
    const double nx = fg[0], ny = fg[1], ufx = fg[3], ufy = fg[4];
    const double cdx = g.cdx[8 * c + 2 * s], cdy = g.cdx[8 * c + 2 * s + 1];
    double* r = rec + (size_t)f * NREC;
    if (o == kNbWall) {
      // wall density from zero net mass flux (Eq. maxWalldes)
      if (g.type[c] != 1) continue;
      FaceEq<double> e;
      e.load(r);
      const double sg = r[R_SGN], nwx = sg * nx, nwy = sg * ny;
      const double lw = r[R_LAMW], hwn = r[R_HWN], vwx = r[R_VWX], vwy = r[R_VWY];
      double num = 0.0, den = 0.0;
      for (int k = lane; k < g.nv; k += 64) {
        const double vx = g.vx[k], vy = g.vy[k];
        const double wn = exact_wn(vx, vy, ufx, ufy, nwx, nwy);
        Local<D> Lh, Lb;
        local_data<D>(g, h, hinf, c, nbc, G, k, Lh);
        local_data<D>(g, b, binf, c, nbc, G, k, Lb);
        double Ih, Ib;
        interface_avg<double>(e, D, 3 - D, vx, vy, vx - ufx, vy - ufy, Lh.v0 + Lh.gx * cdx + Lh.gy * cdy,
                              Lb.v0 + Lb.gx * cdx + Lb.gy * cdy, Lh.gx, Lh.gy, Lb.gx, Lb.gy, Ih, Ib);
        const double cx = vx - vwx, cy = (D == 2) ? vy - vwy : 0.0;
        const double hw = hwn * exp(-lw * (cx * cx + cy * cy));
        num += (wn > 0.0) ? g.wk[k] * wn * Ih : 0.0;
        den += (wn < 0.0) ? g.wk[k] * wn * hw : 0.0;
      }
      num = wave_sum(num);
      den = wave_sum(den);
      if (lane == 0) r[R_RHOW] = -num / den;
      continue;
    }
    // moments of the upwind interface data about the mean velocity of the sides
    const int Lc = (s & 1) ? c : o, Rc = (s & 1) ? o : c;
    double sx, sy;
    {
      double WL[4], WR[4];
      for (int m = 0; m < nw; ++m) {
        WL[m] = (Lc >= 0) ? W[(size_t)Lc * nw + m] : (Lc == kNbFar ? g.winf[m] : W[(size_t)c * nw + m]);
        WR[m] = (Rc >= 0) ? W[(size_t)Rc * nw + m] : (Rc == kNbFar ? g.winf[m] : W[(size_t)c * nw + m]);
      }
      sx = 0.5 * (WL[1] / WL[0] + WR[1] / WR[0]);
      sy = (D == 2) ? 0.5 * (WL[2] / WL[0] + WR[2] / WR[0]) : 0.0;
    }
    double m0 = 0, m1x = 0, m1y = 0, m2 = 0, pxx = 0, pxy = 0, pyy = 0, m3x = 0, m3y = 0;
    for (int k = lane; k < g.nv; k += 64) {
      const double vx = g.vx[k], vy = g.vy[k];
      const double wn = exact_wn(vx, vy, ufx, ufy, nx, ny);
      Local<D> Lh, Lb;
      local_data<D>(g, h, hinf, c, nbc, G, k, Lh);
      local_data<D>(g, b, binf, c, nbc, G, k, Lb);
      const double hc = Lh.v0 + Lh.gx * cdx + Lh.gy * cdy;
      const double bc = Lb.v0 + Lb.gx * cdx + Lb.gy * cdy;
      double ho, bo, t0, t1;
      if (o >= 0) {
        neighbour_recon<D>(g, h, hinf, o, s, Lh.nbv[s], Lh.v0, k, ho, t0, t1);
        neighbour_recon<D>(g, b, binf, o, s, Lb.nbv[s], Lb.v0, k, bo, t0, t1);
      } else {
        ho = (o == kNbFar) ? (double)hinf[k] : Lh.v0;
        bo = (o == kNbFar) ? (double)binf[k] : Lb.v0;
      }
      const double hl = (s & 1) ? hc : ho, hr = (s & 1) ? ho : hc;
      const double bl = (s & 1) ? bc : bo, br = (s & 1) ? bo : bc;
      double fh = (wn > 0.0) ? hl : ((wn < 0.0) ? hr : 0.5 * (hl + hr));
      double fb = (wn > 0.0) ? bl : ((wn < 0.0) ? br : 0.5 * (bl + br));
      const double w = g.wk[k];
      const double cx = vx - sx, cy = (D == 2) ? vy - sy : 0.0;
      const double e = (cx * cx + cy * cy) * fh + fb;
      const double wh = w * fh, we = w * e;
      m0 += wh;
      m1x += wh * cx;
      m2 += we;
      pxx += wh * cx * cx;
      m3x += we * cx;
      if (D == 2) {
        m1y += wh * cy;
        pxy += wh * cx * cy;
        pyy += wh * cy * cy;
        m3y += we * cy;
      }
    }
    m0 = wave_sum(m0); m1x = wave_sum(m1x); m2 = wave_sum(m2); pxx = wave_sum(pxx); m3x = wave_sum(m3x);
    if (D == 2) { m1y = wave_sum(m1y); pxy = wave_sum(pxy); pyy = wave_sum(pyy); m3y = wave_sum(m3y); }
    if (lane != 0) continue;
    // face state from the shifted moments
    const double rho = m0;
    const double dx = m1x / m0, dy = m1y / m0;
    const double ux = sx + dx, uy = sy + dy;
    const double eint = 0.5 * (m2 - (m1x * m1x + m1y * m1y) / m0);
    const double lam = 0.25 * (double)(D + 3 - D) * rho / eint;
    // heat flux about the face velocity: 2q = m3 - 2 P d - d m2 + 2 m0 |d|^2 d
    const double dd = dx * dx + dy * dy;
    double qx = 0.5 * (m3x - 2.0 * (pxx * dx + pxy * dy) - dx * m2 + 2.0 * m0 * dd * dx);
    double qy = 0.5 * (m3y - 2.0 * (pxy * dx + pyy * dy) - dy * m2 + 2.0 * m0 * dd * dy);
    if (D == 1) qy = 0.0;
    r[R_RHO] = rho; r[R_UX] = ux; r[R_UY] = uy; r[R_LAM] = lam; r[R_QX] = qx; r[R_QY] = qy;
    r[R_HN] = rho * pow(lam / kPi, 0.5 * D);
    r[R_SH] = 4.0 * (1.0 - g.pr) * lam * lam / (5.0 * rho);
    double dW[8];
    for (int m = 0; m < 2 * nw; ++m) {
      double gl = (Lc >= 0) ? gW[(size_t)Lc * 8 + m] : 0.0;
      double gr = (Rc >= 0) ? gW[(size_t)Rc * 8 + m] : 0.0;
      dW[m] = 0.5 * (gl + gr);
    }
    expansion(D, rho, ux, uy, lam, ufx, ufy, dW, r + R_AX, r + R_AY, r + R_AT);
    double tq[5];
    time_integrals(dts, inv_tau_of(g, rho, lam), tq);
    for (int m = 0; m < 5; ++m) r[R_T1 + m] = tq[m] / dts;
    r[R_ACT] = 1.0;
    record_derived(r, g.dim, g.nxi, ufx, ufy);
  }
}

// flux: divergence D of field cells, macro flux of the faces the cell owns
// (wall faces also give the wall output)
template <int D, class T, class C>
__global__ __launch_bounds__(256) void k_flux(Dev g, const T* __restrict__ h, const T* __restrict__ b,
                                              const double* __restrict__ rec, T* __restrict__ Dh,
                                              T* __restrict__ Db, double* __restrict__ F,
                                              double* __restrict__ wall) {
  const int c = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
  const int lane = threadIdx.x & 63;
  if (c >= g.ncell || g.type[c] == 0) return;
  const T* hinf = (const T*)g.finf_h;
  const T* binf = (const T*)g.finf_b;
  const bool field = (g.type[c] == 1);
  const double ivol = 1.0 / g.vol[c];
  const int nw = D + 2;
  int nbc[2 * D], fc[2 * D], oc[2 * D];
  bool act[2 * D], own[2 * D];
#pragma unroll
  for (int s = 0; s < 2 * D; ++s) {
    nbc[s] = g.nb[4 * c + s];
    fc[s] = g.cf[4 * c + s];
    own[s] = owns(g, c, s, fc[s]);
    act[s] = fc[s] >= 0 && g.fact[fc[s]] && (field || own[s]);
    oc[s] = act[s] ? g.fcell[2 * fc[s] + ((s & 1) ? 1 : 0)] : kNbMiss;
  }
  const double* G = g.G + 4 * c;
  double acc[2 * D][4];
#pragma unroll
  for (int s = 0; s < 2 * D; ++s)
#pragma unroll
    for (int m = 0; m < 4; ++m) acc[s][m] = 0.0;
  for (int k0 = 0; k0 < g.nv; k0 += 64) {
    const int k = k0 + lane;
    const bool kin = k < g.nv;
    const int kk = kin ? k : g.nv - 1;
    const double vx = g.vx[kk], vy = g.vy[kk], wk = kin ? g.wk[kk] : 0.0;
    Local<D> Lh, Lb;
    local_data<D>(g, h, hinf, c, nbc, G, kk, Lh);
    local_data<D>(g, b, binf, c, nbc, G, kk, Lb);
    double dh = 0.0, db = 0.0;
#pragma unroll
    for (int s = 0; s < 2 * D; ++s) {
      if (!act[s]) continue;
      const int f = fc[s], o = oc[s];
      const double* r = rec + (size_t)f * NREC;
      const double* fg = g.fgeo + (size_t)f * 8;
      const double cdx = g.cdx[8 * c + 2 * s], cdy = g.cdx[8 * c + 2 * s + 1];
      double fh, fb;  // flux along the face normal
      if (o == kNbWall) {
        const double sg = r[R_SGN];
        const double wn = exact_wn(vx, vy, fg[3], fg[4], sg * fg[0], sg * fg[1]);
        FaceEq<C> e;
        e.load(r);
        C Ih, Ib;
        interface_avg<C>(e, D, 3 - D, (C)vx, (C)vy, (C)(vx - fg[3]), (C)(vy - fg[4]),
                         (C)(Lh.v0 + Lh.gx * cdx + Lh.gy * cdy), (C)(Lb.v0 + Lb.gx * cdx + Lb.gy * cdy),
                         (C)Lh.gx, (C)Lh.gy, (C)Lb.gx, (C)Lb.gy, Ih, Ib);
        const double cx = vx - r[R_VWX], cy = (D == 2) ? vy - r[R_VWY] : 0.0;
        const double hw = r[R_RHOW] * r[R_HWN] * exp(-r[R_LAMW] * (cx * cx + cy * cy));
        const double rt = (double)(3 - D) * 0.5 / r[R_LAMW];
        fh = (wn > 0.0) ? sg * wn * (double)Ih : ((wn < 0.0) ? sg * wn * hw : 0.0);
        fb = (wn > 0.0) ? sg * wn * (double)Ib : ((wn < 0.0) ? sg * wn * rt * hw : 0.0);
      } else {
        const double wn = exact_wn(vx, vy, fg[3], fg[4], fg[0], fg[1]);
        const bool upc = (wn > 0.0) == ((s & 1) != 0);  // the upwind side is c
        double vh, vb, ghx, ghy, gbx, gby;
        if (o >= 0) {
          double oh, ob, ohx, ohy, obx, oby;
          neighbour_recon<D>(g, h, hinf, o, s, Lh.nbv[s], Lh.v0, kk, oh, ohx, ohy);
          neighbour_recon<D>(g, b, binf, o, s, Lb.nbv[s], Lb.v0, kk, ob, obx, oby);
          vh = upc ? Lh.v0 + Lh.gx * cdx + Lh.gy * cdy : oh;
          vb = upc ? Lb.v0 + Lb.gx * cdx + Lb.gy * cdy : ob;
          ghx = upc ? Lh.gx : ohx; ghy = upc ? Lh.gy : ohy;
          gbx = upc ? Lb.gx : obx; gby = upc ? Lb.gy : oby;
        } else {
          const double gh0 = (o == kNbFar) ? (double)hinf[kk] : Lh.v0;
          const double gb0 = (o == kNbFar) ? (double)binf[kk] : Lb.v0;
          vh = upc ? Lh.v0 + Lh.gx * cdx + Lh.gy * cdy : gh0;
          vb = upc ? Lb.v0 + Lb.gx * cdx + Lb.gy * cdy : gb0;
          ghx = upc ? Lh.gx : 0.0; ghy = upc ? Lh.gy : 0.0;
          gbx = upc ? Lb.gx : 0.0; gby = upc ? Lb.gy : 0.0;
        }
        FaceEq<C> e;
        e.load(r);
        C Ih, Ib;
        interface_avg<C>(e, D, 3 - D, (C)vx, (C)vy, (C)(vx - fg[3]), (C)(vy - fg[4]), (C)vh, (C)vb,
                         (C)ghx, (C)ghy, (C)gbx, (C)gby, Ih, Ib);
        fh = (wn != 0.0) ? wn * (double)Ih : 0.0;
        fb = (wn != 0.0) ? wn * (double)Ib : 0.0;
      }
      fh = kin ? fh : 0.0;
      fb = kin ? fb : 0.0;
      const double sig = (s & 1) ? 1.0 : -1.0;  // +1 if the face normal points out of c
      dh -= sig * fg[2] * fh * ivol;
      db -= sig * fg[2] * fb * ivol;
      if (own[s]) {
        acc[s][0] += wk * fh;
        acc[s][1] += wk * vx * fh;
        if (D == 2) acc[s][2] += wk * vy * fh;
        acc[s][D + 1] += wk * 0.5 * ((vx * vx + vy * vy) * fh + fb);
      }
    }
    if (kin) {
      Dh[(size_t)c * g.nv + k] = field ? (T)dh : (T)0;
      Db[(size_t)c * g.nv + k] = field ? (T)db : (T)0;
    }
  }
#pragma unroll
  for (int s = 0; s < 2 * D; ++s) {
    if (!own[s] || !act[s]) continue;
    const int f = fc[s];
    double v[4];
#pragma unroll
    for (int m = 0; m < D + 2; ++m) v[m] = wave_sum(acc[s][m]);
    if (lane == 0) {
      if (F) for (int m = 0; m < nw; ++m) F[(size_t)f * nw + m] = v[m];
      if (wall && oc[s] == kNbWall) {
        const double* r = rec + (size_t)f * NREC;
        double* o = wall + (size_t)f * (nw + 1);
        o[0] = r[R_RHOW];
        for (int m = 0; m < nw; ++m) o[1 + m] = r[R_SGN] * v[m];
      }
    }
  }
}

// ------------------------------------------------------------------------
// row-group march (2D).  A workgroup holds RG core rows and the rows just
// below and above them (RG + 2 wavefronts) of one block, for one chunk of 64
// velocities, and marches along i.  At column x every wavefront reconstructs
// the next cell of its row once (values and gradients of h and b into LDS);
// then the core wavefronts evaluate the i-face (x|x+1) of their row and every
// wavefront below the top halo the j-face above its row at column x; in
// flux mode the core rows then gather the divergence of cell x.  Face
// moments (MODE 0) and macro fluxes (MODE 1) are written as per-chunk
// partial sums, reduced over chunks by the finalize kernels in a fixed order.
// Face records are wave-uniform and come through the scalar cache, their
// lines requested one column ahead.
// ------------------------------------------------------------------------
constexpr int kMomP = 9;   // partial values per face and chunk, MODE 0
constexpr int kFluxP = 4;  // MODE 1

template <class C>
struct LD6 {
  C hv, hx, hy, bv, bx, by;
};

template <class T, class C>
__device__ __forceinline__ C cfetch(const T* __restrict__ f, const T* __restrict__ finf, int code, C self, int nv,
                                    int k) {
  if (code >= 0) return (C)f[(size_t)code * nv + k];
  if (code == kNbFar) return (C)finf[k];
  return self;
}

// reciprocal of a nonzero value of normal range: the hardware estimate, in
// double refined by two Newton steps (relative error near 1 ulp)
template <class C>
__device__ __forceinline__ C recip_nr(C d);
template <>
__device__ __forceinline__ double recip_nr<double>(double d) {
  double r = __builtin_amdgcn_rcp(d);
  r = fma(r, fma(-d, r, 1.0), r);
  r = fma(r, fma(-d, r, 1.0), r);
  return r;
}
template <>
__device__ __forceinline__ float recip_nr<float>(float d) { return __builtin_amdgcn_rcpf(d); }

// van Leer slope (s1 |s2| + |s1| s2) / (|s1| + |s2|), which is
// 2 s1 s2 / (s1 + s2) where the one-sided slopes agree in sign and 0 where
// they do not; slopes whose sum is below the normal range (f in the far
// tails) also give 0, so the reciprocal never overflows
template <class C>
__device__ __forceinline__ C vanleer(C vlo, C v0, C vhi) {
  const C s1 = v0 - vlo, s2 = vhi - v0;
  const C sum = s1 + s2;
  const C tiny = (sizeof(C) == 8) ? C(1e-300) : C(1e-36);
  const C vl = C(2) * s1 * s2 * recip_nr<C>(sum);
  return (s1 * s2 <= C(0) || !(fabs(sum) >= tiny)) ? C(0) : vl;
}
// slope of a cell between neighbours of codes lo and hi: none across a
// missing neighbour or between two walls, one-sided next to a wall, else
// van Leer
template <class C>
__device__ __forceinline__ C climit(int lo, int hi, C vlo, C v0, C vhi) {
  if (lo == kNbMiss || hi == kNbMiss) return C(0);
  if (lo == kNbWall && hi == kNbWall) return C(0);
  if (lo == kNbWall) return vhi - v0;
  if (hi == kNbWall) return v0 - vlo;
  return vanleer<C>(vlo, v0, vhi);
}

// value and physical gradient of one component at cell c (codes nbc)
template <class T, class C>
__device__ __forceinline__ void cell_recon(const Dev& g, const T* __restrict__ f, const T* __restrict__ finf, int c,
                                           const int* nbc, const double* G, int k, C& v, C& gx, C& gy) {
  v = (C)f[(size_t)c * g.nv + k];
  C n0 = cfetch<T, C>(f, finf, nbc[0], v, g.nv, k), n1 = cfetch<T, C>(f, finf, nbc[1], v, g.nv, k);
  C n2 = cfetch<T, C>(f, finf, nbc[2], v, g.nv, k), n3 = cfetch<T, C>(f, finf, nbc[3], v, g.nv, k);
  C si = climit<C>(nbc[0], nbc[1], n0, v, n1);
  C sj = climit<C>(nbc[2], nbc[3], n2, v, n3);
  gx = (C)G[0] * si + (C)G[1] * sj;
  gy = (C)G[2] * si + (C)G[3] * sj;
}

// data of one side of a face: reconstructed value at the face and gradient
template <class C>
struct Side {
  C hv, bv, hx, hy, bx, by;
};

template <class T, class C>
__device__ __forceinline__ Side<C> side_from_cell(const Dev& g, const LD6<C>& L, int c, int slot) {
  Side<C> S;
  C dx = (C)g.cdx[8 * c + 2 * slot], dy = (C)g.cdx[8 * c + 2 * slot + 1];
  S.hv = L.hv + L.hx * dx + L.hy * dy;
  S.bv = L.bv + L.bx * dx + L.by * dy;
  S.hx = L.hx; S.hy = L.hy; S.bx = L.bx; S.by = L.by;
  return S;
}

// ghost side (far field or copy of the interior cell c with data L), zero slope
template <class T, class C>
__device__ __forceinline__ Side<C> side_ghost(const Dev& g, const LD6<C>& L, int code, int k) {
  Side<C> S;
  const T* hinf = (const T*)g.finf_h;
  const T* binf = (const T*)g.finf_b;
  S.hv = (code == kNbFar) ? (C)hinf[k] : L.hv;
  S.bv = (code == kNbFar) ? (C)binf[k] : L.bv;
  S.hx = S.hy = S.bx = S.by = C(0);
  return S;
}

// lane-held tables: lane l of a wavefront holds entry l of a record; a
// wave-uniform entry is read back with two lane reads, an int32 entry (low
// word) with one
__device__ __forceinline__ double rec_at(double v, int l) { return lane_read(v, l); }
__device__ __forceinline__ int rec_int(double v, int l) { return __builtin_amdgcn_readlane(__double2loint(v), l); }

// scalar-cache prefetch of the records of two faces: one word of each
// 64-byte line of the face record (NREC doubles, 64-byte aligned) that the
// march reads per velocity (lines 0, 2-6: state, time integrals, wall
// fields, moment shift, interface polynomials; line 1 holds the slope and
// time coefficients, which enter only through the polynomials) and of its
// packed geometry (kFpN doubles, 32-byte aligned: two lines).  The words are
// only kept alive (sgpr_keep) so that the loads are issued; a missing face
// (-1) touches face 0.
constexpr int kRecLines = 6;
constexpr int kRecLine[kRecLines] = {0, 2, 3, 4, 5, 6};
constexpr int kTouch = kRecLines + 2;
__device__ __forceinline__ void face_touch(cdouble* rec, cdouble* fpl,
                                           int f0, int f1, int (&t)[2 * kTouch]) {
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int fq = __builtin_amdgcn_readfirstlane(q == 0 ? f0 : f1);
    const int fs = (fq < 0) ? 0 : fq;
    cint* rr = (cint*)(rec + (size_t)fs * NREC);
    cint* pp = (cint*)(fpl + (size_t)fs * kFpN);
#pragma unroll
    for (int m = 0; m < kRecLines; ++m) t[kTouch * q + m] = rr[16 * kRecLine[m]];
    t[kTouch * q + kRecLines] = pp[0];
    t[kTouch * q + kRecLines + 1] = pp[2 * kFpN - 1];
  }
}
__device__ __forceinline__ void sgpr_keep(const int (&t)[2 * kTouch]) {
  asm volatile("" ::"s"(t[0]), "s"(t[1]), "s"(t[2]), "s"(t[3]), "s"(t[4]), "s"(t[5]), "s"(t[6]), "s"(t[7]),
               "s"(t[8]), "s"(t[9]), "s"(t[10]), "s"(t[11]), "s"(t[12]), "s"(t[13]), "s"(t[14]), "s"(t[15]));
}
static_assert(NREC * 8 == 7 * 64 && R_PH / 8 == 5 && (R_KB + 1) <= 56 && R_SX / 8 == 4 && R_T1 / 8 == 2 &&
                  R_SGN / 8 == 3 && R_RHOW / 8 == 3 && kFpN * 8 <= 96,
              "face_touch covers the record lines read per velocity, geometry in 2");

template <int RG, class T, class C, int MODE>
__device__ __forceinline__ void march_body(int BX, int BY, int BZ, const Dev& g, cint* binfo, int nchunk,
                                           const T* __restrict__ h, const T* __restrict__ b, cdouble* rec,
                                           cdouble* fpl, double* __restrict__ part, T* __restrict__ Dh,
                                           T* __restrict__ Db) {
  constexpr int NW = RG + 2;
  // reconstructions of two columns, raw values of one column per row for
  // the j-neighbours, j-face fluxes of two columns (flux pass; rows 0..RG
  // evaluate j-faces).  Face records and geometry are read through the
  // scalar cache (uniform addresses, read-only), prefetched one column ahead.
  // Two reconstruction slots suffice with one barrier per column because the
  // only reconstruction a wavefront reads from another row is the one written
  // in the same column step (the j-face of the column just reconstructed).
  __shared__ LD6<C> lds[2][NW][64];
  __shared__ C pub[2][NW][2][64];
  __shared__ C jfl[(MODE == 1) ? 2 : 1][RG + 1][2][64];
  cint* bi = binfo + 8 * BZ;
  const int ni = bi[0], nj = bi[1], c0 = bi[2], per_i = bi[3], per_j = bi[4];
  const int j0 = BY * RG;
  if (j0 >= nj) return;  // whole workgroup
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int chunk = BX;
  const int k = chunk * 64 + lane;
  const bool kin = k < g.nv;
  const int kk = kin ? k : g.nv - 1;
  const double vx = g.vx[kk], vy = g.vy[kk];
  const double wk = kin ? g.wk[kk] : 0.0;
  const C finh = (C)((const T*)g.finf_h)[kk];
  const C finb = (C)((const T*)g.finf_b)[kk];
  // wrapping without integer division (offsets are a few cells; the loops
  // run more than once only for blocks narrower than the stencil)
  auto wrap_row = [&](int j) -> int {
    if (j >= 0 && j < nj) return j;
    if (!per_j) return -1;
    while (j < 0) j += nj;
    while (j >= nj) j -= nj;
    return j;
  };
  auto col = [&](int x) -> int {  // column in the block, or -1
    if (x >= 0 && x < ni) return x;
    if (!per_i) return -1;
    while (x < 0) x += ni;
    while (x >= ni) x -= ni;
    return x;
  };
  // this wavefront's row (periodic wrap for the halo rows), the row beyond
  // it for the two halo wavefronts, the row above (for the j-face of a
  // wavefront whose own row is outside the block)
  const int jr = wrap_row(j0 - 1 + w);
  const int jo = (jr < 0) ? -1 : (w == 0) ? wrap_row(j0 - 2) : (w == RG + 1) ? wrap_row(j0 + RG + 1) : -1;
  const int jh = wrap_row(j0 + w);
  const bool core = (w >= 1) && (w <= RG) && (j0 - 1 + w < nj);
  const bool jface = (w <= RG) && (j0 - 1 + w < nj);  // evaluates the j-face above its row
  const int prow = (jr >= 0) ? jr : jh;              // row of the packed cell records it reads
  auto cell = [&](int x, int j) -> int { return c0 + x + ni * j; };
  // this lane's entry in column 0 of the rows it reads (a column xw is
  // xw * nv further on); per-lane offsets keep the scalar registers for the
  // face records
  const size_t nv = (size_t)g.nv;
  const size_t o_r = (size_t)cell(0, jr < 0 ? 0 : jr) * nv + kk;
  const size_t o_o = (size_t)cell(0, jo < 0 ? 0 : jo) * nv + kk;
  const size_t o_p = (size_t)cell(0, prow < 0 ? 0 : prow) * kCpN + ((lane < kCpN) ? lane : 0);
  // raw values of wrapped column xw (-1: outside the block) of this row or of
  // the row beyond it
  auto raw_r = [&](int xw, C& vh, C& vb) {
    if (jr < 0 || xw < 0) { vh = C(0); vb = C(0); return; }
    vh = (C)h[o_r + (size_t)xw * nv];
    vb = (C)b[o_r + (size_t)xw * nv];
  };
  auto raw_o = [&](int xw, C& vh, C& vb) {
    if (jo < 0 || xw < 0) { vh = C(0); vb = C(0); return; }
    vh = (C)h[o_o + (size_t)xw * nv];
    vb = (C)b[o_o + (size_t)xw * nv];
  };
  auto slot = [](int x) -> int { return x & 1; };
  // packed cell record of wrapped column xw of row prow (lane l: entry l),
  // zeros outside the block
  auto cplan_at = [&](int xw) -> double {
    if (prow < 0 || xw < 0) return __hiloint2double(0, (lane == kCpType) ? 0 : -1);
    return (lane < kCpN) ? g.cplan[o_p + (size_t)(xw * kCpN)] : 0.0;
  };
  // i-face (x|x+1) of a core row from the cell record of column x (of
  // column 0 for the seam face x = -1), and j-face above (x, jr) from the
  // record of column x; -1 where there is none
  const bool icore = core && jr >= 0;
  auto iface_id = [&](int x, double cpx, double cp0) -> int {
    if (icore && x >= -1 && x < ni) return (x >= 0) ? rec_int(cpx, kCpFace + 1) : rec_int(cp0, kCpFace + 0);
    return -1;
  };
  auto jface_id = [&](int x, double cpx) -> int {
    if (jface && x >= 0 && x < ni) return (jr >= 0) ? rec_int(cpx, kCpFace + 3) : rec_int(cpx, kCpFace + 2);
    return -1;
  };

  // side data at a face from the reconstruction of a cell and the offset
  // from its centroid to the face centre
  auto side_at = [](const LD6<C>& L, double dx, double dy) -> Side<C> {
    Side<C> S;
    S.hv = L.hv + L.hx * (C)dx + L.hy * (C)dy;
    S.bv = L.bv + L.bx * (C)dx + L.by * (C)dy;
    S.hx = L.hx; S.hy = L.hy; S.bx = L.bx; S.by = L.by;
    return S;
  };
  // raw values of this row: window (x, x+1, x+2) and the next column in
  // flight; the outer row of a halo wavefront at x+1 and x+2
  C a0h, a0b, a1h, a1b, a2h, a2b, p_h, p_b, oc_h, oc_b, on_h, on_b;
  // reconstruction of column x + 1 (window centre) into LDS
  auto recon = [&](int x1, int xw1, double cp) {
    if (jr < 0) return;
    if (xw1 < 0) return;
    if (rec_int(cp, kCpType) == 0) return;
    int nbc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) nbc[q] = rec_int(cp, kCpNb + q);
    double G[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) G[q] = rec_at(cp, kCpG + q);
    const int pp = x1 & 1;
    auto nbv = [&](int code, C cellv, C finv, C self) -> C {
      return (code >= 0) ? cellv : ((code == kNbFar) ? finv : self);
    };
    const C lo_h = (w == 0) ? oc_h : pub[pp][(w == 0) ? 0 : w - 1][0][lane];
    const C lo_b = (w == 0) ? oc_b : pub[pp][(w == 0) ? 0 : w - 1][1][lane];
    const C hi_h = (w == RG + 1) ? oc_h : pub[pp][(w == RG + 1) ? RG + 1 : w + 1][0][lane];
    const C hi_b = (w == RG + 1) ? oc_b : pub[pp][(w == RG + 1) ? RG + 1 : w + 1][1][lane];
    C sih, sjh, sib, sjb;
    if ((nbc[0] | nbc[1] | nbc[2] | nbc[3]) >= 0) {
      // four neighbouring cells (most of the field): van Leer in both
      // directions, no boundary codes to test
      sih = vanleer<C>(a0h, a1h, a2h);
      sjh = vanleer<C>(lo_h, a1h, hi_h);
      sib = vanleer<C>(a0b, a1b, a2b);
      sjb = vanleer<C>(lo_b, a1b, hi_b);
    } else {
      sih = climit<C>(nbc[0], nbc[1], nbv(nbc[0], a0h, finh, a1h), a1h, nbv(nbc[1], a2h, finh, a1h));
      sjh = climit<C>(nbc[2], nbc[3], nbv(nbc[2], lo_h, finh, a1h), a1h, nbv(nbc[3], hi_h, finh, a1h));
      sib = climit<C>(nbc[0], nbc[1], nbv(nbc[0], a0b, finb, a1b), a1b, nbv(nbc[1], a2b, finb, a1b));
      sjb = climit<C>(nbc[2], nbc[3], nbv(nbc[2], lo_b, finb, a1b), a1b, nbv(nbc[3], hi_b, finb, a1b));
    }
    LD6<C> L;
    L.hv = a1h;
    L.hx = (C)G[0] * sih + (C)G[1] * sjh;
    L.hy = (C)G[2] * sih + (C)G[3] * sjh;
    L.bv = a1b;
    L.bx = (C)G[0] * sib + (C)G[1] * sjb;
    L.by = (C)G[2] * sib + (C)G[3] * sjb;
    lds[slot(x1)][w][lane] = L;
  };
  auto ghost = [&](const LD6<C>& L, int code) -> Side<C> {
    Side<C> S;
    S.hv = (code == kNbFar) ? finh : L.hv;
    S.bv = (code == kNbFar) ? finb : L.bv;
    S.hx = S.hy = S.bx = S.by = C(0);
    return S;
  };
  // upwind interface data of a face between sides sl (low) and sh (high)
  // with normal (nx, ny) and mesh velocity (ux, uy)
  auto face_eval = [&](auto r, auto fp, const Side<C>& sl, const Side<C>& sh, double* facc,
                       double* mom) -> void {
    const double nx = fp[kFpN0], ny = fp[kFpN0 + 1], ux = fp[kFpU], uy = fp[kFpU + 1];
    const double wn = exact_wn(vx, vy, ux, uy, nx, ny);
    if (MODE == 0) {
      // moments of the upwind data about the mean velocity of the sides
      const double sx = r[R_SX], sy = r[R_SY];
      double fh = (wn > 0.0) ? (double)sl.hv : ((wn < 0.0) ? (double)sh.hv : 0.5 * ((double)sl.hv + (double)sh.hv));
      double fb = (wn > 0.0) ? (double)sl.bv : ((wn < 0.0) ? (double)sh.bv : 0.5 * ((double)sl.bv + (double)sh.bv));
      const double cx = vx - sx, cy = vy - sy;
      const double e = (cx * cx + cy * cy) * fh + fb;
      const double wh = wk * fh, we = wk * e;
      mom[0] = wh; mom[1] = wh * cx; mom[2] = wh * cy; mom[3] = we; mom[4] = wh * cx * cx;
      mom[5] = wh * cx * cy; mom[6] = wh * cy * cy; mom[7] = we * cx; mom[8] = we * cy;
      return;
    }
    const bool up_low = wn > 0.0;
    const Side<C>& u = up_low ? sl : sh;
    C Ih, Ib;
    interface_poly<C>(r, (C)(vx - r[R_UX]), (C)(vy - r[R_UY]), (C)(vx - ux), (C)(vy - uy), u.hv, u.bv, u.hx, u.hy,
                      u.bx, u.by, Ih, Ib);
    double fh = (wn != 0.0) ? wn * (double)Ih : 0.0;
    double fb = (wn != 0.0) ? wn * (double)Ib : 0.0;
    fh = kin ? fh : 0.0;
    fb = kin ? fb : 0.0;
    facc[0] = fh;
    facc[1] = fb;
    mom[0] = wk * fh; mom[1] = wk * vx * fh; mom[2] = wk * vy * fh;
    mom[3] = wk * 0.5 * ((vx * vx + vy * vy) * fh + fb);
  };
  // wall face seen from the interior cell c (slot s) with data L: MODE 0
  // gives the numerator and denominator of the wall density (Eq. rhow)
  auto wall_eval = [&](auto r, auto fp, bool low, const LD6<C>& L, double* facc,
                       double* mom) -> void {
    const double sg = r[R_SGN];
    const double fg[5] = {fp[kFpN0], fp[kFpN0 + 1], fp[kFpS], fp[kFpU], fp[kFpU + 1]};
    const double wn = exact_wn(vx, vy, fg[3], fg[4], sg * fg[0], sg * fg[1]);
    const Side<C> S = side_at(L, low ? fp[kFpDL] : fp[kFpDR], low ? fp[kFpDL + 1] : fp[kFpDR + 1]);
    C Ih, Ib;
    interface_poly<C>(r, (C)(vx - r[R_UX]), (C)(vy - r[R_UY]), (C)(vx - fg[3]), (C)(vy - fg[4]), S.hv, S.bv, S.hx,
                      S.hy, S.bx, S.by, Ih, Ib);
    if (MODE == 0) {
      const double cx = vx - r[R_VWX], cy = vy - r[R_VWY];
      const double hw = r[R_HWN] * exp(-r[R_LAMW] * (cx * cx + cy * cy));
      mom[0] = (wn > 0.0) ? wk * wn * (double)Ih : 0.0;
      mom[1] = (wn < 0.0) ? wk * wn * hw : 0.0;
      return;
    }
    const double cx = vx - r[R_VWX], cy = vy - r[R_VWY];
    const double hw = r[R_RHOW] * r[R_HWN] * exp(-r[R_LAMW] * (cx * cx + cy * cy));
    const double rt = 0.5 / r[R_LAMW];
    double fh = (wn > 0.0) ? sg * wn * (double)Ih : ((wn < 0.0) ? sg * wn * hw : 0.0);
    double fb = (wn > 0.0) ? sg * wn * (double)Ib : ((wn < 0.0) ? sg * wn * rt * hw : 0.0);
    fh = kin ? fh : 0.0;
    fb = kin ? fb : 0.0;
    facc[0] = fh;
    facc[1] = fb;
    mom[0] = wk * fh; mom[1] = wk * vx * fh; mom[2] = wk * vy * fh;
    mom[3] = wk * 0.5 * ((vx * vx + vy * vy) * fh + fb);
  };
  // chunk partials of the faces evaluated at one column: the i-face (fiw)
  // and the j-face (fjw), each written when this wavefront owns it (else
  // -1), reduced over the 64 lanes together
  auto write_partials = [&](int fiw, const double* mi, int fjw, const double* mj) {
    if (fiw < 0 && fjw < 0) return;
    if (MODE == 0) {
      double v[16], u[2];
#pragma unroll
      for (int q = 0; q < kMomP; ++q) v[q] = mi[q];
#pragma unroll
      for (int q = 0; q < 7; ++q) v[kMomP + q] = mj[q];
      u[0] = mj[7]; u[1] = mj[8];
      multi_sum<16>(v, lane);
      multi_sum<2>(u, lane);
      const int qv = lane >> 2;  // value of v[0]
      if ((lane & 3) == 0) {
        if (qv < kMomP) { if (fiw >= 0) part[((size_t)chunk * g.nface + fiw) * kMomP + qv] = v[0]; }
        else if (fjw >= 0) part[((size_t)chunk * g.nface + fjw) * kMomP + (qv - kMomP)] = v[0];
      }
      if ((lane & 31) == 0 && fjw >= 0) part[((size_t)chunk * g.nface + fjw) * kMomP + 7 + (lane >> 5)] = u[0];
    } else {
      // MODE 1 reduces each face as soon as it is evaluated (see below)
      (void)mi; (void)mj;
    }
  };
  // MODE 1: the four macro-flux partials of one face, reduced at once
  auto write_flux = [&](int fw, double* m) {
    if (fw < 0) return;
    multi_sum<4>(m, lane);
    if ((lane & 15) == 0) part[((size_t)chunk * g.nface + fw) * kFluxP + (lane >> 4)] = m[0];
  };
  // march: step x reconstructs column x + 1, then evaluates the i-face
  // (x|x+1) and the j-face above column x + 1 and, in flux mode, gathers the
  // divergence of column x (its j-faces come from the previous step).  Ahead
  // of use, in registers: raw values (two columns), packed cell records
  // (three columns); in the scalar cache: face records (one column).
  // wrapped columns x + 1, x + 3 and x + 4 of the march step x, advanced
  // by one column per step
  int c1 = col(-1), c2 = col(0), c3 = col(1), c4 = col(2);
  raw_r(col(-2), a0h, a0b);
  raw_r(c1, a1h, a1b);
  raw_r(c2, a2h, a2b);
  raw_r(c3, p_h, p_b);
  raw_o(c1, oc_h, oc_b);
  raw_o(c2, on_h, on_b);
  pub[1][w][0][lane] = a1h;  // column -1
  pub[1][w][1][lane] = a1b;
  // cell records of columns -2 .. 1 and 0
  double cp0c = cplan_at(col(-2)), cp1 = cplan_at(c1), cp2 = cplan_at(c2), cp3 = cplan_at(c3);
  const double cpz = cp2;
  lds_barrier();
  double fi_m1[2] = {0.0, 0.0}, fj_m1[2] = {0.0, 0.0};
  // the records of the next column's faces are requested after this
  // column's faces and waited for before the next column's: one round trip
  // per column instead of several dependent ones per face
  int touched[2 * kTouch] = {};
  // divergence of cell (x, jr) of a core row from the i-faces (x-1|x) and
  // (x|x+1), the j-face above (this row, evaluated one column step earlier)
  // and the j-face below (evaluated by the row beneath, handed over in LDS)
  auto divergence = [&](int x, double cp, const double* fi_lo, const double* fi_hi, const double* fj_up) {
    if (!(core && jr >= 0 && x >= 0 && kin)) return;
    const int c = cell(x, jr);
    double dh = 0.0, db = 0.0;
    if (rec_int(cp, kCpType) == 1) {
      const double ivol = rec_at(cp, kCpIvol);
      const double S0 = rec_at(cp, kCpS), S1 = rec_at(cp, kCpS + 1), S2 = rec_at(cp, kCpS + 2),
                   S3 = rec_at(cp, kCpS + 3);
      const double bh = (double)jfl[x & 1][w - 1][0][lane], bb = (double)jfl[x & 1][w - 1][1][lane];
      dh = -ivol * (-S0 * fi_lo[0] + S1 * fi_hi[0] - S2 * bh + S3 * fj_up[0]);
      db = -ivol * (-S0 * fi_lo[1] + S1 * fi_hi[1] - S2 * bb + S3 * fj_up[1]);
    }
    Dh[(size_t)c * g.nv + k] = (T)dh;
    Db[(size_t)c * g.nv + k] = (T)db;
  };
  // one column step; for a column of known parity P (0 or 1) the LDS slot,
  // hand-over and publication indices become constants
  auto column = [&](int xin, auto par) __attribute__((always_inline)) {
    constexpr int P = decltype(par)::value;
    const int x = (P < 0) ? xin : ((xin & ~1) | P);
    // registers: cell records cp0c .. cp3 of columns x .. x+3 (cp3 in flight)
    recon(x + 1, c1, cp1);
    // publish column x + 2 of this row, advance the windows
    pub[x & 1][w][0][lane] = a2h;
    pub[x & 1][w][1][lane] = a2b;
    a0h = a1h; a0b = a1b; a1h = a2h; a1b = a2b; a2h = p_h; a2b = p_b;
    raw_r(c4, p_h, p_b);
    oc_h = on_h; oc_b = on_b;
    raw_o(c3, on_h, on_b);
    const double cfac = cp0c;  // column x
    cp0c = cp1; cp1 = cp2; cp2 = cp3;
    cp3 = cplan_at(c4);
    {
      // column x + 5: the next in the block, or wrapped (periodic), or -1
      int cn = c4 + 1;
      cn = (cn >= ni) ? 0 : cn;
      cn = per_i ? cn : ((x + 5 < ni) ? x + 5 : -1);
      c1 = c2; c2 = c3; c3 = c4; c4 = cn;
    }
    lds_barrier();
    if (x >= -1) {
      const int sx0 = slot(x), sx1 = slot(x + 1);
      double fi_cur[2] = {0.0, 0.0}, fj_cur[2] = {0.0, 0.0};
      constexpr int NM = (MODE == 0) ? kMomP : kFluxP;
      double mi[NM], mj[NM];
#pragma unroll
      for (int q = 0; q < NM; ++q) { mi[q] = 0.0; mj[q] = 0.0; }
      int fiw = -1, fjw = -1;
      // the i-face (x|x+1) and the j-face above column x + 1, whose
      // reconstructions were written in this column step
      int fid[2];
      fid[0] = iface_id(x, cfac, cpz);
      fid[1] = jface_id(x + 1, cp0c);  // cp0c: column x + 1
      sgpr_keep(touched);
      // q = 0 the i-face (x|x+1) of a core row, q = 1 the j-face above
      // (x + 1, jr) for the bottom halo and core rows
      auto face_q = [&](int q) {
        const int f = (q == 0) ? fid[0] : fid[1];
        if (f < 0) return;
        const int fu = __builtin_amdgcn_readfirstlane(f);
        cdouble* r = rec + (size_t)fu * NREC;
        // the face geometry, read field by field where it is used (its lines
        // were requested one column ahead)
        cdouble* fp = fpl + (size_t)fu * kFpN;
        if (__builtin_amdgcn_readfirstlane(tab_int(fp[kFpAct])) == 0) return;
        const int L = __builtin_amdgcn_readfirstlane(tab_int(fp[kFpL]));
        const int R = __builtin_amdgcn_readfirstlane(tab_int(fp[kFpR]));
        // owner: the low cell, or the cell of a boundary face; a periodic
        // seam i-face (x = -1) is written by the high end of the row; the
        // bottom halo writes only the block's lower boundary j-face
        const bool owner = ((q == 0) ? (x >= 0) : (w >= 1)) || (L < 0);
        const LD6<C>& lo = lds[(q == 0) ? sx0 : sx1][w][lane];
        const LD6<C>& hi = lds[sx1][(q == 0) ? w : w + 1][lane];
        double fc[2] = {0.0, 0.0}, mom[NM];
#pragma unroll
        for (int m = 0; m < NM; ++m) mom[m] = 0.0;
        if (L == kNbWall || R == kNbWall) {
          wall_eval(r, fp, L != kNbWall, (L == kNbWall) ? hi : lo, fc, mom);
        } else {
          // the low side of the seam face (x = -1) is cell ni-1, staged as column -1
          Side<C> sl, sh;
          if ((L | R) >= 0) {
            // interior face (most faces): both sides reconstructed
            sl = side_at(lo, fp[kFpDL], fp[kFpDL + 1]);
            sh = side_at(hi, fp[kFpDR], fp[kFpDR + 1]);
          } else {
            sl = (L >= 0) ? side_at(lo, fp[kFpDL], fp[kFpDL + 1]) : ghost(hi, L);
            sh = (R >= 0) ? side_at(hi, fp[kFpDR], fp[kFpDR + 1]) : ghost(lo, R);
          }
          face_eval(r, fp, sl, sh, fc, mom);
        }
        if (MODE == 1) write_flux(owner ? f : -1, mom);
        if (q == 0) {
          fi_cur[0] = fc[0]; fi_cur[1] = fc[1];
          if constexpr (MODE == 0) {
            if (owner) fiw = f;
#pragma unroll
            for (int m = 0; m < NM; ++m) mi[m] = mom[m];
          }
        } else {
          fj_cur[0] = fc[0]; fj_cur[1] = fc[1];
          if constexpr (MODE == 0) {
            if (owner) fjw = f;
#pragma unroll
            for (int m = 0; m < NM; ++m) mj[m] = mom[m];
          }
        }
      };
      face_q(0);
      face_q(1);
      if (MODE == 1 && x + 1 < ni && jface) {
        jfl[(x + 1) & 1][w][0][lane] = (C)fj_cur[0];
        jfl[(x + 1) & 1][w][1][lane] = (C)fj_cur[1];
      }
      if (MODE == 0) write_partials(fiw, mi, fjw, mj);
      if (MODE == 1) divergence(x, cfac, fi_m1, fi_cur, fj_m1);
      fi_m1[0] = fi_cur[0]; fi_m1[1] = fi_cur[1];
      fj_m1[0] = fj_cur[0]; fj_m1[1] = fj_cur[1];
      face_touch(rec, fpl, iface_id(x + 1, cp0c, cpz), jface_id(x + 2, cp1), touched);  // cp1: column x + 2
    }
  };
  if constexpr (sizeof(C) == 8) {
    // two columns per iteration: the loop-carried windows rotate by two
    // and the parities are constants (2-3 % on the FP64 passes)
    for (int x = -2; x < ni; x += 2) {
      column(x, std::integral_constant<int, 0>{});
      if (x + 1 < ni) column(x + 1, std::integral_constant<int, 1>{});
    }
  } else {
    // one column per iteration: the FP32 passes stay within 128 VGPRs, so
    // that two 6-row workgroups share a CU
    for (int x = -2; x < ni; ++x) column(x, std::integral_constant<int, -1>{});
  }
}
template <int RG, class T, class C, int MODE>
__global__ __launch_bounds__(64 * (RG + 2)) void k_march(Dev g, const int* __restrict__ binfo, int nchunk,
                                                         const T* __restrict__ h, const T* __restrict__ b,
                                                         const double* __restrict__ rec,
                                                         const double* __restrict__ fpl,
                                                         double* __restrict__ part, T* __restrict__ Dh,
                                                         T* __restrict__ Db) {
  march_body<RG, T, C, MODE>(blockIdx.x, blockIdx.y, blockIdx.z, g, (cint*)binfo, nchunk, h, b, (cdouble*)rec,
                             (cdouble*)fpl, part, Dh, Db);
}

// face records from the chunk partials of the face moments (interior and
// ghost faces) and the wall density (wall faces)
__device__ __forceinline__ void face_fin_body(int BX, const Dev& g, double dts, int nchunk,
                                              const double* __restrict__ part, const double* __restrict__ W,
                                              const double* __restrict__ gW, double* __restrict__ rec) {
  int f = BX * blockDim.x + threadIdx.x;
  if (f >= g.nface || !g.fact[f]) return;
  const int L = g.fcell[2 * f], R = g.fcell[2 * f + 1];
  double m[kMomP];
  for (int q = 0; q < kMomP; ++q) m[q] = 0.0;
  // chunk order kept; unrolled so that several chunks' loads are in flight
#pragma unroll 8
  for (int ch = 0; ch < nchunk; ++ch) {
    const double* p = part + ((size_t)ch * g.nface + f) * kMomP;
#pragma unroll
    for (int q = 0; q < kMomP; ++q) m[q] += p[q];
  }
  double* r = rec + (size_t)f * NREC;
  if (L == kNbWall || R == kNbWall) {
    r[R_RHOW] = -m[0] / m[1];
    return;
  }
  const double sx = r[R_SX], sy = r[R_SY];
  const double m0 = m[0], m1x = m[1], m1y = m[2], m2 = m[3], pxx = m[4], pxy = m[5], pyy = m[6], m3x = m[7],
               m3y = m[8];
  const double rho = m0;
  const double dx = m1x / m0, dy = m1y / m0;
  const double ux = sx + dx, uy = sy + dy;
  const double eint = 0.5 * (m2 - (m1x * m1x + m1y * m1y) / m0);
  const double lam = 0.75 * rho / eint;
  const double dd = dx * dx + dy * dy;
  const double qx = 0.5 * (m3x - 2.0 * (pxx * dx + pxy * dy) - dx * m2 + 2.0 * m0 * dd * dx);
  const double qy = 0.5 * (m3y - 2.0 * (pxy * dx + pyy * dy) - dy * m2 + 2.0 * m0 * dd * dy);
  r[R_RHO] = rho; r[R_UX] = ux; r[R_UY] = uy; r[R_LAM] = lam; r[R_QX] = qx; r[R_QY] = qy;
  r[R_HN] = rho * (lam / kPi);
  r[R_SH] = 4.0 * (1.0 - g.pr) * lam * lam / (5.0 * rho);
  double dW[8];
  for (int q = 0; q < 8; ++q) {
    double gl = (L >= 0) ? gW[(size_t)L * 8 + q] : 0.0;
    double gr = (R >= 0) ? gW[(size_t)R * 8 + q] : 0.0;
    dW[q] = 0.5 * (gl + gr);
  }
  const double* fg = g.fgeo + (size_t)f * 8;
  expansion(2, rho, ux, uy, lam, fg[3], fg[4], dW, r + R_AX, r + R_AY, r + R_AT);
  double tq[5];
  time_integrals(dts, inv_tau_of(g, rho, lam), tq);
  for (int q = 0; q < 5; ++q) r[R_T1 + q] = tq[q] / dts;
  r[R_ACT] = 1.0;
  record_derived(r, 2, g.nxi, fg[3], fg[4]);
}
__global__ void k_face_fin(Dev g, double dts, int nchunk, const double* __restrict__ part,
                           const double* __restrict__ W, const double* __restrict__ gW, double* __restrict__ rec) {
  face_fin_body(blockIdx.x, g, dts, nchunk, part, W, gW, rec);
}

// macro flux per face (and the wall output) from the chunk partials
__device__ __forceinline__ void flux_fin_body(int BX, const Dev& g, int nchunk, const double* __restrict__ part,
                                              const double* __restrict__ rec, double* __restrict__ F,
                                              double* __restrict__ wall) {
  int f = BX * blockDim.x + threadIdx.x;
  if (f >= g.nface || !g.fact[f]) return;
  double m[kFluxP] = {0, 0, 0, 0};
  // chunk order kept; unrolled so that several chunks' loads are in flight
#pragma unroll 8
  for (int ch = 0; ch < nchunk; ++ch) {
    const double* p = part + ((size_t)ch * g.nface + f) * kFluxP;
#pragma unroll
    for (int q = 0; q < kFluxP; ++q) m[q] += p[q];
  }
  if (F) for (int q = 0; q < kFluxP; ++q) F[(size_t)f * 4 + q] = m[q];
  const int L = g.fcell[2 * f], R = g.fcell[2 * f + 1];
  if (wall && (L == kNbWall || R == kNbWall)) {
    const double* r = rec + (size_t)f * NREC;
    double* o = wall + (size_t)f * 5;
    o[0] = r[R_RHOW];
    for (int q = 0; q < 4; ++q) o[1 + q] = r[R_SGN] * m[q];
  }
}
__global__ void k_flux_fin(Dev g, int nchunk, const double* __restrict__ part, const double* __restrict__ rec,
                           double* __restrict__ F, double* __restrict__ wall) {
  flux_fin_body(blockIdx.x, g, nchunk, part, rec, F, wall);
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
__device__ __forceinline__ void step7_body(int BX, const Dev& g, int mode, const T* __restrict__ h,
                                           const T* __restrict__ b, const double* __restrict__ crec,
                                           const double* __restrict__ Wp, double* __restrict__ W,
                                           double* __restrict__ q, double* __restrict__ mrec) {
  int c = BX * 4 + (threadIdx.x >> 6);
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
  // mode 2, and the receptors in mode 1 (their W is the interpolated one,
  // unchanged by the step): heat flux of f about the velocity of W, so that
  // a receptor that turns into a field cell starts from q^n of its f^n
  if (mode == 2 || (mode == 1 && !step)) {
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
  bool finite = true;
  for (int m = 0; m < g.nw; ++m) {
    w[m] = wp[m] + (fm[m] - gm[m]);
    finite = finite && isfinite(w[m]);
  }
  // a non-physical or non-finite state is reported through the status word
  if (!finite || !physical_state(g.dim, w)) raise_status(g.status, kStatusNonPhys);
  double r2, ux, uy, l2;
  prim_of(g, w, r2, ux, uy, l2);
  double qx, qy;
  heat_from_record(M, ux, uy, g.dim, qx, qy);
  q[(size_t)c * g.dim] = qx;
  if (g.dim == 2) q[(size_t)c * g.dim + 1] = qy;
}
template <class T>
__global__ __launch_bounds__(256) void k_step7(Dev g, int mode, const T* __restrict__ h,
                                               const T* __restrict__ b, const double* __restrict__ crec,
                                               const double* __restrict__ Wp, double* __restrict__ W,
                                               double* __restrict__ q, double* __restrict__ mrec) {
  step7_body<T>(blockIdx.x, g, mode, h, b, crec, Wp, W, q, mrec);
}

// per-cell record from W (or W') and the heat flux (given, or from a moment
// record shifted to the velocity of W), the micro diagonal base for the
// physical step dt, and the micro face coefficients
__device__ __forceinline__ void cellrec_body(int BX, const Dev& g, double dt, const double* __restrict__ W,
                                             const double* __restrict__ q, const double* __restrict__ mrec,
                                             double* __restrict__ crec) {
  int c = BX * blockDim.x + threadIdx.x;
  if (c >= g.ncell) return;
  crec[(size_t)c * NCREC + C_FLD] = (g.type[c] == 1) ? 1.0 : 0.0;
  if (g.type[c] == 0) return;
  double rho, ux, uy, lam;
  prim_of(g, W + (size_t)c * g.nw, rho, ux, uy, lam);
  double qx, qy;
  if (mrec) heat_from_record(mrec + (size_t)c * NMREC, ux, uy, g.dim, qx, qy);
  else { qx = q[(size_t)c * g.dim]; qy = (g.dim == 2) ? q[(size_t)c * g.dim + 1] : 0.0; }
  double* r = crec + (size_t)c * NCREC;
  r[C_RHO] = rho; r[C_UX] = ux; r[C_UY] = uy; r[C_LAM] = lam; r[C_QX] = qx; r[C_QY] = qy;
  r[C_HN] = rho * pow(lam / kPi, 0.5 * g.dim);
  r[C_SH] = 4.0 * (1.0 - g.pr) * lam * lam / (5.0 * rho);
  double it = inv_tau_of(g, rho, lam);
  r[C_ITAU] = it;
  r[C_D0] = 1.0 / g.dtp[c] + 1.0 / dt + 0.5 * it;
  for (int m = 0; m < 12; ++m) r[C_GEO + m] = g.mgeo[(size_t)c * 12 + m];
}
__global__ void k_cellrec(Dev g, double dt, const double* __restrict__ W, const double* __restrict__ q,
                          const double* __restrict__ mrec, double* __restrict__ crec) {
  cellrec_body(blockIdx.x, g, dt, W, q, mrec, crec);
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
__device__ __forceinline__ void interp_body(int BX, const Dev& g, int nrec, const int* __restrict__ rec,
                                            const int* __restrict__ ptr, const int* __restrict__ don,
                                            const double* __restrict__ wt, T* __restrict__ h, T* __restrict__ b,
                                            double* __restrict__ W, double* __restrict__ q) {
  int r = BX * 4 + (threadIdx.x >> 6);
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
template <class T>
__global__ __launch_bounds__(256) void k_interp(Dev g, int nrec, const int* __restrict__ rec,
                                                const int* __restrict__ ptr, const int* __restrict__ don,
                                                const double* __restrict__ wt, T* __restrict__ h,
                                                T* __restrict__ b, double* __restrict__ W,
                                                double* __restrict__ q) {
  interp_body<T>(blockIdx.x, g, nrec, rec, ptr, don, wt, h, b, W, q);
}

// ------------------------------------------------------------------------
// macro LU-SGS (Eq. dualTimeStepping_macro)
// ------------------------------------------------------------------------
// spectral radius per face from W^s
__device__ __forceinline__ void gamma_body(int BX, const Dev& g, const double* __restrict__ W,
                                           double* __restrict__ gam) {
  int f = BX * blockDim.x + threadIdx.x;
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
__global__ void k_gamma(Dev g, const double* __restrict__ W, double* __restrict__ gam) {
  gamma_body(blockIdx.x, g, W, gam);
}

// macro record per cell (computed in parallel before the sweep):
//   [0..3] residual R, [4] 1/D (LU-SGS diagonal), [5] 1/(4|Omega|),
//   per slot s at 8 + 14 s: neighbour state W_nb (4), its Euler flux
//   F_E(W_nb; n_out, U_f) (4), n_out (2), U_f.n_out, S, S Gamma, field flag
constexpr int kMacRec = 64;
constexpr int kMacSlot = 14;

__device__ __forceinline__ void euler_flux_n(int dim, const double* w, double nx, double ny, double un, double* o);

__device__ __forceinline__ void macro_prep_body(int BX, const Dev& g, double dt, const double* __restrict__ W,
                                                const double* __restrict__ Wn, const double* __restrict__ F,
                                                const double* __restrict__ Fn, const double* __restrict__ gam,
                                                double* __restrict__ mac) {
  int c = BX * blockDim.x + threadIdx.x;
  if (c >= g.ncell) return;
  const int nw = g.nw;
  double* M = mac + (size_t)c * kMacRec;
  for (int m = 0; m < kMacRec; ++m) M[m] = 0.0;
  if (g.type[c] != 1) return;
  const double ivol = 1.0 / g.vol[c];
  double r[4] = {0, 0, 0, 0}, sg = 0.0;
  for (int m = 0; m < nw; ++m) r[m] = -(W[(size_t)c * nw + m] - Wn[(size_t)c * nw + m]) / dt;
  for (int s = 0; s < 2 * g.dim; ++s) {
    int f = g.cf[4 * c + s];
    double* P = M + 8 + kMacSlot * s;
    if (f < 0) continue;
    const double* fg = g.fgeo + (size_t)f * 8;
    const double S = fg[2];
    const double sig = (s & 1) ? 1.0 : -1.0;
    for (int m = 0; m < nw; ++m)
      r[m] -= 0.5 * ivol * sig * S * (F[(size_t)f * nw + m] + Fn[(size_t)f * nw + m]);
    sg += S * gam[f];
    const int o = g.nb[4 * c + s];
    const double nx = sig * fg[0], ny = sig * fg[1];
    const double un = fg[3] * nx + fg[4] * ny;
    const bool fld = (o >= 0) && g.type[o] == 1;
    const double* wn = fld ? W + (size_t)o * nw : W + (size_t)c * nw;
    double wv[4] = {0, 0, 0, 0}, fe[4] = {0, 0, 0, 0};
    for (int m = 0; m < nw; ++m) wv[m] = wn[m];
    euler_flux_n(g.dim, wv, nx, ny, un, fe);
    for (int m = 0; m < 4; ++m) { P[m] = wv[m]; P[4 + m] = fe[m]; }
    P[8] = nx; P[9] = ny; P[10] = un;
    P[11] = fld ? S : 0.0;
    P[12] = fld ? S * gam[f] : 0.0;
    P[13] = fld ? 1.0 : 0.0;
  }
  for (int m = 0; m < 4; ++m) M[m] = r[m];
  const double Dg = 1.0 / g.dtp[c] + 1.0 / dt + 0.25 * ivol * sg;
  M[4] = 1.0 / Dg;
  M[5] = 0.25 * ivol;
  M[6] = Dg;
  M[7] = 0.0;
}
__global__ void k_macro_prep(Dev g, double dt, const double* __restrict__ W, const double* __restrict__ Wn,
                             const double* __restrict__ F, const double* __restrict__ Fn,
                             const double* __restrict__ gam, double* __restrict__ mac) {
  macro_prep_body(blockIdx.x, g, dt, W, Wn, F, Fn, gam, mac);
}

// ALE Euler flux difference F_E(W + dW) - F_E(W) along n with mesh velocity U
__device__ __forceinline__ void euler_flux4(int dim, int nxi, double w0, double w1, double w2, double w3,
                                            double nx, double ny, double ux, double uy, double* o) {
  double rho = w0, vx = w1 / rho, vy = (dim == 2) ? w2 / rho : 0.0;
  double wE = (dim == 2) ? w3 : w2;
  double e = wE - 0.5 * rho * (vx * vx + vy * vy);
  double p = 2.0 * e / (double)(dim + nxi);  // rho/(2 lam)
  double th = (vx - ux) * nx + ((dim == 2) ? (vy - uy) * ny : 0.0);
  o[0] = rho * th;
  o[1] = w1 * th + p * nx;
  if (dim == 2) { o[2] = w2 * th + p * ny; o[3] = wE * th + p * (vx * nx + vy * ny); }
  else o[2] = wE * th + p * vx * nx;
}

// ALE Euler flux of w along n with the mesh normal velocity un = U.n
__device__ __forceinline__ void euler_flux_n(int dim, const double* w, double nx, double ny, double un, double* o) {
  const double ir = 1.0 / w[0];
  const double vx = w[1] * ir, vy = (dim == 2) ? w[2] * ir : 0.0;
  const double wE = w[dim + 1];
  const double p = 2.0 / 3.0 * (wE - 0.5 * w[0] * (vx * vx + vy * vy));  // rho/(2 lam), D + N_xi = 3
  const double vn = vx * nx + ((dim == 2) ? vy * ny : 0.0);
  const double th = vn - un;
  o[0] = w[0] * th;
  o[1] = w[1] * th + p * nx;
  if (dim == 2) { o[2] = w[2] * th + p * ny; o[3] = wE * th + p * vn; }
  else o[2] = wE * th + p * vn;
}

__device__ __forceinline__ void euler_dflux(int dim, int nxi, const double* W, const double* dW, double nx,
                                            double ny, double ux, double uy, double* out) {
  double f1[4], f0[4];
  euler_flux4(dim, nxi, W[0] + dW[0], W[1] + dW[1], W[2] + dW[2], (dim == 2) ? W[3] + dW[3] : 0.0, nx, ny,
              ux, uy, f1);
  euler_flux4(dim, nxi, W[0], W[1], W[2], (dim == 2) ? W[3] : 0.0, nx, ny, ux, uy, f0);
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
// macro sweep: one workgroup per block, one thread per row j.  The next
// hyperplane's inputs (residual, diagonal, neighbour states and face data)
// are loaded before the current hyperplane is computed, so their latency
// overlaps the computation and the barrier.
// macro sweep: one workgroup per block, one thread per row j, hyperplane
// order.  The inputs of the next hyperplane (macro record: residual or dW*,
// 1/D, and the two structural couplings) are requested before the current
// hyperplane is computed and no load address depends on a loaded value; the
// couplings across periodic seams are copied to LDS at the start.
struct MacroRow {
  bool ok;
  int c;
  double base[4], iD, ivd;
  double nb[2][kMacSlot];
};

// forward (bwd = 0): base = residual from the record, lower couplings;
// backward: base = dW* (`dws`), upper couplings
template <int D>
__device__ __forceinline__ void macro_row_load(const double* __restrict__ mac, const double* __restrict__ dws,
                                               int bwd, int ni, int nj, int c0, int j, int h, MacroRow& M) {
  int i = h - j;
  M.ok = (j < nj) && (i >= 0) && (i < ni);
  if (!M.ok) return;
  const int c = c0 + i + ni * j;
  M.c = c;
  const double* R = mac + (size_t)c * kMacRec;
  M.iD = R[4];
  M.ivd = R[5];
#pragma unroll
  for (int m = 0; m < 4; ++m) M.base[m] = bwd ? ((m < D + 2) ? dws[(size_t)c * (D + 2) + m] : 0.0) : R[m];
  const int s0 = bwd ? 1 : 0, s1 = bwd ? 3 : 2;
#pragma unroll
  for (int m = 0; m < kMacSlot; ++m) {
    M.nb[0][m] = R[8 + kMacSlot * s0 + m];
    M.nb[1][m] = (D == 2) ? R[8 + kMacSlot * s1 + m] : 0.0;
  }
}

// S (F_E(W_nb + x) - F_E(W_nb) - Gamma x) added to acc
template <int D>
__device__ __forceinline__ void macro_couple(const double* P, const double* x, double* acc) {
  if (P[13] == 0.0) return;
  double w[4], fe[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) w[m] = P[m] + ((m < D + 2) ? x[m] : 0.0);
  euler_flux_n(D, w, P[8], P[9], P[10], fe);
#pragma unroll
  for (int m = 0; m < D + 2; ++m) acc[m] += P[11] * (fe[m] - P[4 + m]) - P[12] * x[m];
}

// LDS doubles of the macro sweep: hand-off [2][NT][4], periodic-j values
// [ni][4], seam couplings [2][nj][14] (periodic i) and [2][ni][14] (periodic j)
size_t macro_lds(int nt, int max_ni, int max_nj, int any_pi, int any_pj) {
  return sizeof(double) * (size_t)(2 * nt * 4 + (any_pj ? 4 * max_ni + 2 * kMacSlot * max_ni : 0) +
                                   (any_pi ? 2 * kMacSlot * max_nj : 0));
}

// rows of records in flight in the one-wavefront macro sweep
#ifndef UGKS_MACRO_RING
#define UGKS_MACRO_RING 3
#endif

// NTB: the launch's thread bound (64 for blocks up to 64 cells tall: one
// wavefront, whose ring of prefetched rows then has the register file to
// itself; 512 otherwise)
template <int D, int NTB>
__device__ __forceinline__ void macro_sweep_body(int BX, const Dev& g, const int* __restrict__ binfo,
                                                 const double* __restrict__ W, const double* __restrict__ mac,
                                                 double* __restrict__ dWs, double* __restrict__ dW,
                                                 double* __restrict__ Wp, double* __restrict__ rpart, int max_ni,
                                                 int max_nj, int any_pi, int any_pj) {
  extern __shared__ double msm[];
  const int* bi = binfo + 8 * BX;
  const int ni = bi[0], nj = bi[1], c0 = bi[2], pi = bi[3], pj = bi[4];
  const int j = threadIdx.x;
  const int NT = blockDim.x;
  constexpr int nw = D + 2;
  double* hand = msm;                                              // [2][NT][4]
  double* pjb = msm + 2 * NT * 4;                                  // [ni][4]
  double* sjp = pjb + (any_pj ? 4 * max_ni : 0);                   // [2][ni][14]
  double* sip = sjp + (any_pj ? 2 * kMacSlot * max_ni : 0);        // [2][nj][14]
  (void)max_nj; (void)any_pi;
  // seam couplings: periodic i (cell (ni-1, j) slot 1, cell (0, j) slot 0),
  // periodic j (cell (i, nj-1) slot 3, cell (i, 0) slot 2)
  if (pi && j < nj)
    for (int m = 0; m < kMacSlot; ++m) {
      sip[(0 * nj + j) * kMacSlot + m] = mac[(size_t)(c0 + ni - 1 + ni * j) * kMacRec + 8 + kMacSlot * 1 + m];
      sip[(1 * nj + j) * kMacSlot + m] = mac[(size_t)(c0 + ni * j) * kMacRec + 8 + kMacSlot * 0 + m];
    }
  if (D == 2 && pj)
    for (int i = j; i < ni; i += NT)
      for (int m = 0; m < kMacSlot; ++m) {
        sjp[(0 * ni + i) * kMacSlot + m] = mac[(size_t)(c0 + i + ni * (nj - 1)) * kMacRec + 8 + kMacSlot * 3 + m];
        sjp[(1 * ni + i) * kMacSlot + m] = mac[(size_t)(c0 + i) * kMacRec + 8 + kMacSlot * 2 + m];
      }
  // residual norm over the block's field cells (the record of any other
  // cell holds zeros)
  double rs[4] = {0, 0, 0, 0};
  if (j < nj)
    for (int i = 0; i < ni; ++i) {
      const double* R = mac + (size_t)(c0 + i + ni * j) * kMacRec;
#pragma unroll
      for (int m = 0; m < nw; ++m) rs[m] += R[m] * R[m];
    }
  for (int m = 0; m < 4; ++m) rs[m] = wave_sum(rs[m]);
  // per-wave sums combined in a fixed order (the hand-off buffer is free
  // until the forward sweep starts; all LDS of this kernel is dynamic)
  if ((j & 63) == 0) for (int m = 0; m < 4; ++m) hand[(j >> 6) * 4 + m] = rs[m];
  __syncthreads();
  if (j == 0) {
    for (int m = 0; m < nw; ++m) {
      double t = 0.0;
      for (int w = 0; w < (NT + 63) / 64; ++w) t += hand[w * 4 + m];
      rpart[(size_t)BX * 4 + m] = t;
    }
  }
  __syncthreads();
  const int H = ni + nj - 1;
  double prev[4] = {0, 0, 0, 0}, cw[4] = {0, 0, 0, 0};
  // forward sweep: (D + L) dW* = R.  The records of hyperplane h + RING - 1
  // are loaded while h is solved (a ring of rows in registers): the sweep is
  // one wavefront per block, so each hyperplane's latency is exposed
  auto fwd_step = [&](int h, const MacroRow& cur) __attribute__((always_inline)) {
    if (!cur.ok) return;
    const int i = h - j, c = cur.c;
    double x[4] = {0, 0, 0, 0};
    if (cur.iD > 0.0) {
      double acc[4] = {0, 0, 0, 0};
      if (i >= 1) macro_couple<D>(cur.nb[0], prev, acc);
      if (D == 2 && j >= 1) macro_couple<D>(cur.nb[1], hand + ((h - 1) & 1) * NT * 4 + (j - 1) * 4, acc);
      if (pi && i == ni - 1 && ni > 1) macro_couple<D>(sip + (0 * nj + j) * kMacSlot, cw, acc);
      if (D == 2 && pj && j == nj - 1 && nj > 1) macro_couple<D>(sjp + (0 * ni + i) * kMacSlot, pjb + 4 * i, acc);
#pragma unroll
      for (int m = 0; m < nw; ++m) x[m] = (cur.base[m] - cur.ivd * acc[m]) * cur.iD;
    }
#pragma unroll
    for (int m = 0; m < nw; ++m) {
      dWs[(size_t)c * nw + m] = x[m];
      prev[m] = x[m];
      if (i == 0) cw[m] = x[m];
      hand[(h & 1) * NT * 4 + j * 4 + m] = x[m];
      if (pj && j == 0) pjb[4 * i + m] = x[m];
    }
  };
  // ring of UGKS_MACRO_RING rows for a one-wavefront launch; of two
  // (prefetch one hyperplane ahead) for the wide launch, whose registers a
  // deeper ring would exceed
  constexpr int RING = (NTB == 64) ? UGKS_MACRO_RING : 2;
  MacroRow ring[RING];
#pragma unroll
  for (int u = 0; u < RING - 1; ++u) macro_row_load<D>(mac, dWs, 0, ni, nj, c0, j, u, ring[u]);
  for (int h0 = 0; h0 < H; h0 += RING) {
#pragma unroll
    for (int u = 0; u < RING; ++u) {
      const int h = h0 + u;
      if (h >= H) break;
      macro_row_load<D>(mac, dWs, 0, ni, nj, c0, j, h + RING - 1, ring[(u + RING - 1) % RING]);
      fwd_step(h, ring[u]);
      lds_barrier();
    }
  }
  for (int m = 0; m < 4; ++m) { prev[m] = 0.0; cw[m] = 0.0; }
  __syncthreads();
  // backward sweep: (D + U) dW = D dW*, the same ring of rows descending
  auto bwd_step = [&](int h, const MacroRow& cur) __attribute__((always_inline)) {
    if (!cur.ok) return;
    const int i = h - j, c = cur.c;
    const bool fld = cur.iD > 0.0;
    double wc[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) wc[m] = (m < nw) ? W[(size_t)c * nw + m] : 0.0;
    double x[4] = {0, 0, 0, 0};
    if (fld) {
      double acc[4] = {0, 0, 0, 0};
      if (i + 1 < ni) macro_couple<D>(cur.nb[0], prev, acc);
      if (D == 2 && j + 1 < nj) macro_couple<D>(cur.nb[1], hand + ((h + 1) & 1) * NT * 4 + (j + 1) * 4, acc);
      if (pi && i == 0 && ni > 1) macro_couple<D>(sip + (1 * nj + j) * kMacSlot, cw, acc);
      if (D == 2 && pj && j == 0 && nj > 1) macro_couple<D>(sjp + (1 * ni + i) * kMacSlot, pjb + 4 * i, acc);
#pragma unroll
      for (int m = 0; m < nw; ++m) x[m] = cur.base[m] - cur.ivd * cur.iD * acc[m];
    }
    // a non-physical predictor keeps the current state
    double wp[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) wp[m] = (m < nw) ? wc[m] + x[m] : 0.0;
    const bool keep = physical_state(D, wp) && fld;
#pragma unroll
    for (int m = 0; m < nw; ++m) {
      dW[(size_t)c * nw + m] = x[m];
      Wp[(size_t)c * nw + m] = wc[m] + (keep ? x[m] : 0.0);  // (a select of wp / wc here goes to scratch)
      prev[m] = x[m];
      if (i == ni - 1) cw[m] = x[m];
      hand[(h & 1) * NT * 4 + j * 4 + m] = x[m];
      if (pj && j == nj - 1) pjb[4 * i + m] = x[m];
    }
  };
#pragma unroll
  for (int u = 0; u < RING - 1; ++u) macro_row_load<D>(mac, dWs, 1, ni, nj, c0, j, H - 1 - u, ring[u]);
  for (int h0 = H - 1; h0 >= 0; h0 -= RING) {
#pragma unroll
    for (int u = 0; u < RING; ++u) {
      const int h = h0 - u;
      if (h < 0) break;
      macro_row_load<D>(mac, dWs, 1, ni, nj, c0, j, h - (RING - 1), ring[(u + RING - 1) % RING]);
      bwd_step(h, ring[u]);
      lds_barrier();
    }
  }
}
template <int D, int NTB>
__global__ __launch_bounds__(NTB) void k_macro_sweep(Dev g, const int* __restrict__ binfo,
                                                     const double* __restrict__ W,
                                                     const double* __restrict__ mac,
                                                     double* __restrict__ dWs, double* __restrict__ dW,
                                                     double* __restrict__ Wp, double* __restrict__ rpart,
                                                     int max_ni, int max_nj, int any_pi, int any_pj) {
  macro_sweep_body<D, NTB>(blockIdx.x, g, binfo, W, mac, dWs, dW, Wp, rpart, max_ni, max_nj, any_pi, any_pj);
}

// L2 norms of the residual: sum the per-block partial sums
__device__ __forceinline__ void resid_body(int nblock, int nw, const double* __restrict__ rpart,
                                           double* __restrict__ out) {
  int m = threadIdx.x;
  if (m >= nw) return;
  double s = 0.0;
  for (int b = 0; b < nblock; ++b) s += rpart[(size_t)b * 4 + m];
  out[m] = sqrt(s);
}
__global__ void k_resid(int nblock, int nw, const double* __restrict__ rpart, double* __restrict__ out) {
  resid_body(nblock, nw, rpart, out);
}

// micro residual r = S - f^s/dt + (D + (f+' - f^s)/tau')/2 of one pair
// (Eq. residual_micro_n+1,s with the stored level-n part S) from the cell's
// equilibrium and rate fields (record r), rounded to the storage type; no
// contraction, so that the residual pass and the forward sweep that forms it
// itself give the same bits
template <class T>
__device__ __forceinline__ void micro_residual(int dim, const double* r, double vx, double vy, double idt,
                                               double f0, double f1, double s0, double s1, double d0,
                                               double d1, double& r0, double& r1) {
#pragma clang fp contract(off)
  const double ux = r[C_UX], uy = r[C_UY], lam = r[C_LAM], qx = r[C_QX], qy = r[C_QY];
  const double hn = r[C_HN], sh = r[C_SH], it = r[C_ITAU];
  const double rt = 0.5 / lam;
  const double cx = vx - ux, cy = (dim == 2) ? vy - uy : 0.0;
  const double c2 = cx * cx + cy * cy;
  const double H = hn * exp(-lam * c2);
  const double B = (double)(3 - dim) * rt * H;
  const double sq = sh * (cx * qx + cy * qy);
  const double tl = 2.0 * lam * c2;
  const double hpl = H + sq * (tl - 2.0 - dim) * H;
  const double bpl = B + sq * (tl - dim) * (double)(3 - dim) * rt * H;
  r0 = (double)(T)(s0 - f0 * idt + 0.5 * (d0 + (hpl - f0) * it));
  r1 = (double)(T)(s1 - f1 * idt + 0.5 * (d1 + (bpl - f1) * it));
}

// the residual pass, written over D: fully parallel, one wavefront per cell,
// the cell record is wave-uniform
template <class T>
__device__ __forceinline__ void micro_rhs_body(int BX, const Dev& g, double dt, const double* __restrict__ crec,
                                               const T* __restrict__ h, const T* __restrict__ b,
                                               const T* __restrict__ Sh, const T* __restrict__ Sb, T* __restrict__ Dh,
                                               T* __restrict__ Db) {
  const int c = __builtin_amdgcn_readfirstlane(BX * 4 + (threadIdx.x >> 6));
  const int lane = threadIdx.x & 63;
  if (c >= g.ncell || g.type[c] != 1) return;
  const double* r = crec + (size_t)c * NCREC;
  const double idt = 1.0 / dt;
  for (int k = lane; k < g.nv; k += 64) {
    const size_t o = (size_t)c * g.nv + k;
    double r0, r1;
    micro_residual<T>(g.dim, r, g.vx[k], (g.dim == 2) ? g.vy[k] : 0.0, idt, (double)h[o], (double)b[o],
                      (double)Sh[o], (double)Sb[o], (double)Dh[o], (double)Db[o], r0, r1);
    Dh[o] = (T)r0;
    Db[o] = (T)r1;
  }
}
template <class T>
__global__ __launch_bounds__(256) void k_micro_rhs(Dev g, double dt, const double* __restrict__ crec,
                                                   const T* __restrict__ h, const T* __restrict__ b,
                                                   const T* __restrict__ Sh, const T* __restrict__ Sb,
                                                   T* __restrict__ Dh, T* __restrict__ Db) {
  micro_rhs_body<T>(blockIdx.x, g, dt, crec, h, b, Sh, Sb, Dh, Db);
}

// micro LU-SGS (Eq. dualTimeStepping_micro): forward and backward sweep of
// one velocity chunk (KC lanes) of one block, R rows per thread slot (rows
// j, j + ceil(nj/R), ...: cells of one hyperplane in different rows are
// independent), in hyperplane order.  Dh/Db hold the residual r on entry (D
// when the forward sweep forms the residual itself, below) and dF* after the
// forward sweep; h, b are updated to f^{s+1} by the backward sweep.
//
// Latency and issue: everything a hyperplane needs from global memory (its
// residual or dF*, h, b, and the cell's coefficient record: face geometry,
// D0 and the field flag) is requested P hyperplanes ahead into a register
// ring, at addresses clamped into the row so that no load is predicated or
// depends on a loaded value.  The record of the next hyperplane is copied
// from the ring to LDS (double buffered) by the KC lanes of its row.  The
// row hand-off buffer has a zero slot below row 0 and above the last row,
// so the couplings need no row tests; results are stored only for cells of
// the block.
//
// Synchronisation per hyperplane: without a periodic seam along j a row's
// neighbours are the rows next to it, so a wavefront depends only on the two
// wavefronts beside it (their edge rows feed its edge rows, and they reuse
// its hand-off slots two hyperplanes later), while rows inside a wavefront
// hand off in the wavefront's own LDS order.  With two rows per thread (rows
// jt and jt + NTR) the first wavefront's second rows and the last
// wavefront's first rows are neighbours too, so the wavefronts form a ring;
// this needs every thread to own distinct rows (NTR * KC a whole number of
// wavefronts).  Each wavefront then publishes its count of finished
// hyperplanes in LDS and waits for its two neighbours to have finished the
// previous one, instead of a workgroup barrier: the wavefront with the least
// progress can always go on, and the wait is bounded (Dev::micro_spin sleeps) so
// that the kernel ends in any case.  A periodic j seam, or threads beyond
// NTR * KC, use the barrier.
//
// With one row per thread and chunks of 8 or 16 velocities (2D) the residual
// is fused into the forward sweep: instead of reading r, written over D by
// k_micro_rhs, it reads D, S and f^s, and the cell's equilibrium and rate
// fields are staged with its record (the residual needs no hand-off value,
// so it is formed before the wait for the neighbour rows).  The 1D sweep (one
// wavefront per chunk) keeps the separate, fully parallel residual pass,
// which would otherwise lengthen its sequential chain.
//
// staged record per row: C_UX .. C_FLD (fused residual) or C_GEO .. C_FLD
constexpr bool micro_fused(int kc, int rows) { return rows == 1 && kc >= 8 && kc <= 16; }
constexpr int micro_rec_lds(int kc, int rows) { return micro_fused(kc, rows) ? 24 : 16; }
constexpr int kMicroProg = 8;   // doubles of LDS for the 16 progress counters

// 1/d for d > 0 of moderate size: hardware estimate and two Newton steps
__device__ __forceinline__ double recip_pos(double d) {
  double r = __builtin_amdgcn_rcp(d);
  r = fma(r, fma(-d, r, 1.0), r);
  r = fma(r, fma(-d, r, 1.0), r);
  return r;
}

template <int D, class T, int KC, int P, int R>
__device__ __forceinline__ void micro_body(int BX, int NBX, int BY, const Dev& g, const int* __restrict__ binfo,
                                           int nslot, const double* __restrict__ crec, T* __restrict__ h,
                                           T* __restrict__ b, T* __restrict__ Dh, T* __restrict__ Db,
                                           const T* __restrict__ Sh, const T* __restrict__ Sb, double dt) {
  extern __shared__ double smem[];
  constexpr bool FUSE = micro_fused(KC, R);
  constexpr int RB = FUSE ? C_UX : C_GEO;       // first staged record entry
  constexpr int NRM = C_FLD + 1 - RB;           // staged entries
  constexpr int RLD = micro_rec_lds(KC, R);     // LDS stride of a staged record
  static_assert(NRM <= RLD, "staged record fits its LDS slot");
  constexpr int NS = (NRM + KC - 1) / KC;       // record entries per lane
  constexpr int OG = C_GEO - RB, OD = C_D0 - RB, OF = C_FLD - RB;
  const int* bi = binfo + 8 * BY;
  const int ni = bi[0], nj = bi[1], c0 = bi[2], pi = bi[3], pj = bi[4];
  const int t = threadIdx.x;
  const int lk = t % KC, jt = t / KC;
  // rows of this thread: jt, jt + NTR, ... (R of them; the cells of one
  // hyperplane in different rows are independent)
  const int NTR = (nslot + R - 1) / R;
  const int nv = g.nv;
  // velocity chunk: chunks that share a 128-byte line of f go to workgroups
  // that the round-robin dispatch places on the same XCD (every 8th
  // workgroup), so each line is fetched once into that XCD's L2
  constexpr int G = (128 / (KC * (int)sizeof(T)) > 1) ? 128 / (KC * (int)sizeof(T)) : 1;
  int chunk = BX;
  if constexpr (G > 1) {
    const int span = 8 * G, base = (chunk / span) * span;
    if (base + span <= NBX) chunk = base + G * (chunk % 8) + (chunk / 8) % G;
  }
  const int k = chunk * KC + lk;
  const bool kin = k < nv;
  const int kk = kin ? k : nv - 1;
  int jr[R], jl[R], cbase[R];
  bool row[R];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    jr[q] = jt + NTR * q;
    row[q] = jr[q] < nj;
    jl[q] = row[q] ? jr[q] : nj - 1;  // rows beyond the block read (not write) the last row's slots
    cbase[q] = c0 + ni * jl[q];       // cell (0, j)
  }
  // LDS: progress counters (16 ints), hand[2][nslot + 2][KC][2] (slot s + 1
  // holds row s), cells[2][nslot][16], pj[ni][KC][2]
  int* prog = (int*)smem;
  double* hand = smem + kMicroProg;
  double* cells = hand + 4 * (nslot + 2) * KC;
  double* pjb = cells + 2 * nslot * RLD;
  auto HND = [&](int p, int s) -> double* { return hand + ((size_t)(p * (nslot + 2) + s) * KC + lk) * 2; };
  auto CEL = [&](int p, int q) -> double* { return cells + (size_t)(p * nslot + jl[q]) * RLD; };
  for (int e = t; e < 4 * (nslot + 2) * KC; e += blockDim.x) hand[e] = 0.0;
  if (t < 2 * kMicroProg) prog[t] = 0;
  const bool p2p = !(D == 2 && pj) && (R == 1 || NTR * KC == (int)blockDim.x);
  const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
  const int nwv = (int)(blockDim.x + 63) >> 6;
  // neighbour wavefronts (-1: none); a ring for two rows per thread
  const int lo_wv = (R == 1) ? wv - 1 : (wv + nwv - 1) % nwv;
  const int hi_wv = (R == 1) ? ((wv + 1 < nwv) ? wv + 1 : -1) : (wv + 1) % nwv;
  int done = 0;  // hyperplanes finished by this wavefront (both sweeps)
  auto prog_of = [&](int v) -> int {
    return __builtin_amdgcn_readfirstlane(__hip_atomic_load(&prog[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
  };
  // before a hyperplane: both neighbour wavefronts have finished `done`
  // If the bound runs out the wavefront goes on (so the kernel always ends)
  // and sets the context's status bit: its results are then not valid and
  // the host reports the failure at its next status check.
  const int spin_limit = g.micro_spin;
  auto wait_neighbours = [&]() {
    bool ready = false;
    for (int spin = 0;; ++spin) {
      const bool lo = (lo_wv < 0) || (lo_wv == wv) || prog_of(lo_wv) >= done;
      const bool hi = (hi_wv < 0) || (hi_wv == wv) || prog_of(hi_wv) >= done;
      ready = lo && hi;
      if (ready || spin >= spin_limit) break;
      __builtin_amdgcn_s_sleep(1);
    }
    if (!ready && (t & 63) == 0) raise_status(g.status, kStatusWait);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
  };
  // after a hyperplane's hand-off writes
  auto publish = [&]() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    ++done;
    if ((t & 63) == 0) __hip_atomic_store(&prog[wv], done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  };
  const double vx = g.vx[kk], vy = (D == 2) ? g.vy[kk] : 0.0;
  const int HH = ni + nj - 1;

  // ring: r (or D when fused) for both components, f^s (backward sweep, and
  // the fused forward sweep), S (fused forward sweep), record entries
  double ra[R][P], rb_[R][P], rf0[R][P], rf1[R][P], rs0[R][P], rs1[R][P];
  double rr[R][P][NS];
  auto issue = [&](int q, int u, int hp, bool bwd) {
    const int i = min(max(hp - jr[q], 0), ni - 1);
    const size_t o = (size_t)(cbase[q] + i) * nv + kk;
    ra[q][u] = (double)Dh[o];
    rb_[q][u] = (double)Db[o];
    if (bwd || FUSE) { rf0[q][u] = (double)h[o]; rf1[q][u] = (double)b[o]; }
    if (FUSE && !bwd) { rs0[q][u] = (double)Sh[o]; rs1[q][u] = (double)Sb[o]; }
    const double* r = crec + (size_t)(cbase[q] + i) * NCREC + RB;
#pragma unroll
    for (int m = 0; m < NS; ++m) rr[q][u][m] = r[min(lk + KC * m, NRM - 1)];  // unpredicated
  };
  auto stage = [&](int q, int u, int p) {
    if (!row[q]) return;
    double* d = CEL(p, q);
#pragma unroll
    for (int m = 0; m < NS; ++m)
      if (lk + KC * m < NRM) d[lk + KC * m] = rr[q][u][m];
  };
  // fused forward sweep: the micro residual of the pair from D, S, f^s and
  // the cell's staged fields, as k_micro_rhs forms it
  const double idt = 1.0 / dt;
  auto resid = [&](int q, int u, int p, double& a0, double& a1) {
    // the staged record starts at entry RB of the cell record
    micro_residual<T>(D, CEL(p, q) - RB, vx, vy, idt, rf0[q][u], rf1[q][u], rs0[q][u], rs1[q][u], ra[q][u],
                      rb_[q][u], a0, a1);
  };
  // one cell of a sweep (nothing is written when (i, j) is outside the block)
  double ph[R], pb[R], chh[R], cbb[R];
#pragma unroll
  for (int q = 0; q < R; ++q) { ph[q] = pb[q] = chh[q] = cbb[q] = 0.0; }
  auto cell = [&](int q, int hp, int p, bool bwd, double a0, double a1, double f0, double f1) {
    const int j = jr[q];
    const int i = hp - j;
    const bool act = row[q] && i >= 0 && i < ni;
    const double* r = CEL(p, q);
    double ts[4];
    double d = r[OD];
#pragma unroll
    for (int s = 0; s < 2 * D; ++s) {
      ts[s] = r[OG + 3 * s] * vx + r[OG + 3 * s + 1] * vy - r[OG + 3 * s + 2];
      d += fmax(ts[s], 0.0);
    }
    const bool fld = act && r[OF] != 0.0;
    // couplings: along i from the row's previous cell (zero before the first
    // cell of the sweep), along j through the hand-off buffer, and across
    // periodic seams
    const int si = bwd ? 1 : 0, sj = bwd ? 3 : 2;
    double w = fmin(ts[si], 0.0);
    double oh = w * ph[q], ob = w * pb[q];
    if (D == 2) {
      const double* hq = HND(p ^ 1, bwd ? jl[q] + 2 : jl[q]);
      w = fmin(ts[sj], 0.0);
      oh += w * hq[0]; ob += w * hq[1];
    }
    const bool seam_i = pi && ni > 1 && i == (bwd ? 0 : ni - 1);
    w = seam_i ? fmin(ts[bwd ? 0 : 1], 0.0) : 0.0;
    oh += w * chh[q]; ob += w * cbb[q];
    if (D == 2 && pj) {
      const bool seam_j = nj > 1 && j == (bwd ? 0 : nj - 1);
      if (seam_j && act) {
        const double* z = pjb + ((size_t)i * KC + lk) * 2;
        w = fmin(ts[bwd ? 2 : 3], 0.0);
        oh += w * z[0]; ob += w * z[1];
      }
    }
    const double id = recip_pos(d);
    double xh = bwd ? a0 - oh * id : (a0 - oh) * id;
    double xb = bwd ? a1 - ob * id : (a1 - ob) * id;
    xh = fld ? xh : 0.0;
    xb = fld ? xb : 0.0;
    if (act) {
      if (fld && kin) {
        const size_t o = (size_t)(cbase[q] + i) * nv + k;
        if (bwd) { h[o] = (T)(f0 + xh); b[o] = (T)(f1 + xb); }
        else { Dh[o] = (T)xh; Db[o] = (T)xb; }
      }
      ph[q] = xh; pb[q] = xb;
      if (i == (bwd ? ni - 1 : 0)) { chh[q] = xh; cbb[q] = xb; }
      double* hq = HND(p, j + 1);
      hq[0] = xh; hq[1] = xb;
      if (D == 2 && pj && j == (bwd ? nj - 1 : 0)) {
        double* z = pjb + ((size_t)i * KC + lk) * 2;
        z[0] = xh; z[1] = xb;
      }
    }
  };

  // ---------------- forward sweep: (D + L) dF* = r ----------------
  // Each ring slot is consumed by its hyperplane and then refilled with the
  // hyperplane P later, so a slot keeps its registers around the loop.  The
  // loop runs whole groups of P hyperplanes; the extra ones (hp >= HH) have
  // no cells in any row.
#pragma unroll
  for (int u = 0; u < P; ++u)
#pragma unroll
    for (int q = 0; q < R; ++q) issue(q, u, u, false);
#pragma unroll
  for (int q = 0; q < R; ++q) stage(q, 0, 0);
  __syncthreads();
  for (int h0 = 0; h0 < HH; h0 += P) {
#pragma unroll
    for (int u = 0; u < P; ++u) {
      const int hp = h0 + u;
      // stage first: the record it waits for was loaded P - 1 hyperplanes
      // ago, and the wait then covers no store of this hyperplane (stores
      // and loads share one in-order counter)
#pragma unroll
      for (int q = 0; q < R; ++q) stage(q, (u + 1) % P, (hp + 1) & 1);
      double a0[R], a1[R];
#pragma unroll
      for (int q = 0; q < R; ++q) {
        if constexpr (FUSE) resid(q, u, hp & 1, a0[q], a1[q]);
        else { a0[q] = ra[q][u]; a1[q] = rb_[q][u]; }
      }
      if (p2p) wait_neighbours();
#pragma unroll
      for (int q = 0; q < R; ++q) cell(q, hp, hp & 1, false, a0[q], a1[q], 0.0, 0.0);
      if (p2p) publish();
#pragma unroll
      for (int q = 0; q < R; ++q) issue(q, u, hp + P, false);
      if (!p2p) lds_barrier();
    }
  }
  // ---------------- backward sweep: (D + U) dF = D dF* ----------------
#pragma unroll
  for (int q = 0; q < R; ++q) { ph[q] = pb[q] = chh[q] = cbb[q] = 0.0; }
#pragma unroll
  for (int u = 0; u < P; ++u)
#pragma unroll
    for (int q = 0; q < R; ++q) issue(q, u, HH - 1 - u, true);
#pragma unroll
  for (int q = 0; q < R; ++q) stage(q, 0, (HH - 1) & 1);
  __syncthreads();
  for (int h0 = HH - 1; h0 >= 0; h0 -= P) {
#pragma unroll
    for (int u = 0; u < P; ++u) {
      const int hp = h0 - u;
#pragma unroll
      for (int q = 0; q < R; ++q) stage(q, (u + 1) % P, (hp - 1) & 1);
      if (p2p) wait_neighbours();
#pragma unroll
      for (int q = 0; q < R; ++q) cell(q, hp, hp & 1, true, ra[q][u], rb_[q][u], rf0[q][u], rf1[q][u]);
      if (p2p) publish();
#pragma unroll
      for (int q = 0; q < R; ++q) issue(q, u, hp - P, true);
      if (!p2p) lds_barrier();
    }
  }
}
template <int D, class T, int KC, int P, int R>
__global__ __launch_bounds__(1024) void k_micro(Dev g, const int* __restrict__ binfo, int nslot,
                                                const double* __restrict__ crec, T* __restrict__ h,
                                                T* __restrict__ b, T* __restrict__ Dh, T* __restrict__ Db,
                                                const T* __restrict__ Sh, const T* __restrict__ Sb, double dt) {
  micro_body<D, T, KC, P, R>(blockIdx.x, (int)gridDim.x, blockIdx.y, g, binfo, nslot, crec, h, b, Dh, Db, Sh, Sb, dt);
}

// ------------------------------------------------------------------------
// host launchers
// ------------------------------------------------------------------------
static inline unsigned nb4(int n) { return (unsigned)((n + 3) / 4); }
static inline unsigned nbl(size_t n, int t) { return (unsigned)((n + t - 1) / t); }

template <int D, class T, class C>
void launch_flux_t(const Dev& g, double dts, const void* h, const void* b, const double* W, const double* q,
                   double* gW, double* rec, void* Dh, void* Db, double* F, double* wall, hipStream_t st,
                   hipEvent_t* ev) {
  k_gradW<<<nbl(g.ncell, 64), 64, 0, st>>>(g, W, gW);
  k_wallprep<<<nbl(g.nface, 64), 64, 0, st>>>(g, dts, W, q, gW, rec);
  if (ev) (void)hipEventRecord(ev[0], st);
  k_face_eq<D, T><<<nb4(g.ncell), 256, 0, st>>>(g, dts, (const T*)h, (const T*)b, W, gW, rec);
  if (ev) { (void)hipEventRecord(ev[1], st); (void)hipEventRecord(ev[2], st); }
  k_flux<D, T, C><<<nb4(g.ncell), 256, 0, st>>>(g, (const T*)h, (const T*)b, rec, (T*)Dh, (T*)Db, F, wall);
  if (ev) (void)hipEventRecord(ev[3], st);
}

// one march pass with RG core rows per workgroup (RG + 2 wavefronts share
// the reconstruction of RG rows)
template <int RG, class T, class C, int MODE>
static void march_pass(const Dev& g, const int* binfo, int max_nj, int nchunk, const void* h, const void* b,
                       const double* W, const double* rec, double* part, void* Dh, void* Db, hipStream_t st) {
  dim3 grid((unsigned)nchunk, (unsigned)((max_nj + RG - 1) / RG), (unsigned)g.nblock);
  (void)W;
  k_march<RG, T, C, MODE><<<grid, 64 * (RG + 2), 0, st>>>(g, binfo, nchunk, (const T*)h, (const T*)b, rec, g.fplan,
                                                           part, (T*)Dh, (T*)Db);
}

template <class T, class C, int MODE>
static void march_rg(int rg, const Dev& g, const int* binfo, int max_nj, int nchunk, const void* h,
                     const void* b, const double* W, const double* rec, double* part, void* Dh, void* Db,
                     hipStream_t st) {
  // 10 core rows: 12 wavefronts, 3 per SIMD, one workgroup per CU in FP64
  if (rg == 6) { march_pass<6, T, C, MODE>(g, binfo, max_nj, nchunk, h, b, W, rec, part, Dh, Db, st); return; }
  if (rg == 10) { march_pass<10, T, C, MODE>(g, binfo, max_nj, nchunk, h, b, W, rec, part, Dh, Db, st); return; }
  march_pass<8, T, C, MODE>(g, binfo, max_nj, nchunk, h, b, W, rec, part, Dh, Db, st);
}

template <class T, class C>
void launch_march_t(const Dev& g, const int* binfo, int max_nj, double dts, const void* h, const void* b,
                    const double* W, const double* q, double* gW, double* rec, double* part, void* Dh, void* Db,
                    double* F, double* wall, hipStream_t st, hipEvent_t* ev) {
  const int nchunk = (g.nv + 63) / 64;
  k_gradW<<<nbl(g.ncell, 64), 64, 0, st>>>(g, W, gW);
  k_wallprep<<<nbl(g.nface, 64), 64, 0, st>>>(g, dts, W, q, gW, rec);
  if (ev) (void)hipEventRecord(ev[0], st);
  march_rg<T, C, 0>(g.rg_eq, g, binfo, max_nj, nchunk, h, b, W, rec, part, Dh, Db, st);
  if (ev) (void)hipEventRecord(ev[1], st);
  k_face_fin<<<nbl(g.nface, 64), 64, 0, st>>>(g, dts, nchunk, part, W, gW, rec);
  if (ev) (void)hipEventRecord(ev[2], st);
  march_rg<T, C, 1>(g.rg_flux, g, binfo, max_nj, nchunk, h, b, W, rec, part, Dh, Db, st);
  if (ev) (void)hipEventRecord(ev[3], st);
  k_flux_fin<<<nbl(g.nface, 64), 64, 0, st>>>(g, nchunk, part, rec, F, wall);
}

void launch_flux(const Dev& g, int prec, const int* binfo, int max_nj, double dts, const void* h, const void* b,
                 const double* W, const double* q, double* gW, double* rec, double* part, void* Dh, void* Db,
                 double* F, double* wall, hipStream_t st, hipEvent_t* ev) {
  if (g.dim == 2) {
    if (prec == 0) launch_march_t<double, double>(g, binfo, max_nj, dts, h, b, W, q, gW, rec, part, Dh, Db, F, wall, st, ev);
    else launch_march_t<float, float>(g, binfo, max_nj, dts, h, b, W, q, gW, rec, part, Dh, Db, F, wall, st, ev);
  } else {
    if (prec == 0) launch_flux_t<1, double, double>(g, dts, h, b, W, q, gW, rec, Dh, Db, F, wall, st, ev);
    else launch_flux_t<1, float, float>(g, dts, h, b, W, q, gW, rec, Dh, Db, F, wall, st, ev);
  }
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

void launch_cellrec(const Dev& g, double dt, const double* W, const double* q, const double* mrec, double* crec,
                    hipStream_t st) {
  k_cellrec<<<nbl(g.ncell, 64), 64, 0, st>>>(g, dt, W, q, mrec, crec);
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

void launch_macro(const Dev& g, const int* binfo, int max_ni, int max_nj, int any_pi, int any_pj, double dt,
                  const double* W, const double* Wn, const double* F, const double* Fn, double* gam, double* R,
                  double* Dg, double* dWs, double* dW, double* Wp, double* rpart, double* resid, hipStream_t st) {
  (void)Dg;
  k_gamma<<<nbl(g.nface, 64), 64, 0, st>>>(g, W, gam);
  k_macro_prep<<<nbl(g.ncell, 64), 64, 0, st>>>(g, dt, W, Wn, F, Fn, gam, R);
  const int nt = ((max_nj + 63) / 64) * 64;
  const size_t lds = macro_lds(nt, max_ni, max_nj, any_pi, any_pj);
  if (g.dim == 2) {
    if (nt == 64)
      k_macro_sweep<2, 64><<<g.nblock, nt, lds, st>>>(g, binfo, W, R, dWs, dW, Wp, rpart, max_ni, max_nj, any_pi,
                                                     any_pj);
    else
      k_macro_sweep<2, 512><<<g.nblock, nt, lds, st>>>(g, binfo, W, R, dWs, dW, Wp, rpart, max_ni, max_nj, any_pi,
                                                      any_pj);
  } else {
    k_macro_sweep<1, 64><<<g.nblock, nt, lds, st>>>(g, binfo, W, R, dWs, dW, Wp, rpart, max_ni, max_nj, any_pi,
                                                   any_pj);
  }
  if (resid) k_resid<<<1, 64, 0, st>>>(g.nblock, g.nw, rpart, resid);
}

// velocity-chunk width of the micro sweep for a block height
#ifndef UGKS_MICRO_DEPTH
#define UGKS_MICRO_DEPTH 3
#endif
static size_t micro_lds_of(int dim, int max_ni, int max_nj, int any_pj, int kc, int rows) {
  const int nslot = (dim == 1) ? 1 : max_nj;
  return sizeof(double) * (size_t)(kMicroProg + 4 * (nslot + 2) * kc + 2 * nslot * micro_rec_lds(kc, rows) +
                                   (any_pj ? 2 * max_ni * kc : 0));
}

// velocity-chunk width KC and rows per thread R of the micro sweep: the
// widest chunk up to kc_max, one row per thread before two, with
// KC * ceil(nj / R) <= 1024 threads and LDS within 160 KiB; kc = 0 when none
// fits
void micro_shape(int dim, int max_ni, int max_nj, int any_pj, int kc_max, int& kc, int& rows) {
  rows = 1;
  if (dim == 1) { kc = 64; return; }
  for (kc = kc_max; kc >= 2; kc >>= 1)
    for (rows = 1; rows <= 2; ++rows)
      if (kc * ((max_nj + rows - 1) / rows) <= 1024 &&
          micro_lds_of(dim, max_ni, max_nj, any_pj, kc, rows) <= 160 * 1024)
        return;
  kc = 0;
  rows = 1;
}

size_t micro_lds(int dim, int max_ni, int max_nj, int any_pj, int kc_max) {
  int kc, rows;
  micro_shape(dim, max_ni, max_nj, any_pj, kc_max, kc, rows);
  if (kc == 0) return (size_t)1 << 40;  // no shape fits
  return micro_lds_of(dim, max_ni, max_nj, any_pj, kc, rows);
}

// ring depth of the sweep: two rows per thread (of FP64 values, or with
// records spread over few lanes) and the fused residual (six values per
// pair) take the registers a third slot would need
template <class T, int KC, int R>
constexpr int micro_depth() {
  return ((R == 2 && (sizeof(T) == 8 || KC <= 4)) || micro_fused(KC, R)) ? 2 : UGKS_MICRO_DEPTH;
}

// ring depth of the launched instance (the kernels' own rule)
template <class T>
static int micro_depth_of(int kc, int rows) {
  switch (kc * 4 + rows) {
    case 64 * 4 + 1: return micro_depth<T, 64, 1>();
    case 16 * 4 + 1: return micro_depth<T, 16, 1>();
    case 16 * 4 + 2: return micro_depth<T, 16, 2>();
    case 8 * 4 + 1: return micro_depth<T, 8, 1>();
    case 8 * 4 + 2: return micro_depth<T, 8, 2>();
    case 4 * 4 + 1: return micro_depth<T, 4, 1>();
    case 4 * 4 + 2: return micro_depth<T, 4, 2>();
    case 2 * 4 + 1: return micro_depth<T, 2, 1>();
    case 2 * 4 + 2: return micro_depth<T, 2, 2>();
    default: return 0;
  }
}

void micro_launch_shape(int dim, int prec, int max_ni, int max_nj, int any_pj, int kc_max, int& kc, int& rows,
                        int& depth, int& fused) {
  micro_shape(dim, max_ni, max_nj, any_pj, kc_max, kc, rows);
  fused = (kc > 0 && micro_fused(kc, rows)) ? 1 : 0;
  depth = (prec == 0) ? micro_depth_of<double>(kc, rows) : micro_depth_of<float>(kc, rows);
}

template <int D, class T, int KC, int R>
static void micro_t(const Dev& g, const int* binfo, int nslot, size_t lds, double dt, const double* crec, void* h,
                    void* b, const void* Sh, const void* Sb,
                    void* Dh, void* Db, hipStream_t st) {
  constexpr int P = micro_depth<T, KC, R>();
  dim3 grid((unsigned)((g.nv + KC - 1) / KC), (unsigned)g.nblock);
  int threads = ((((nslot + R - 1) / R) * KC + 63) / 64) * 64;
  k_micro<D, T, KC, P, R><<<grid, threads, lds, st>>>(g, binfo, nslot, crec, (T*)h, (T*)b, (T*)Dh, (T*)Db,
                                                       (const T*)Sh, (const T*)Sb, dt);
}

template <class T>
static void micro_prec(const Dev& g, const int* binfo, int KC, int R, int nslot, size_t lds, double dt,
                       const double* crec, const void* Sh, const void* Sb,
                       void* h, void* b, void* Dh, void* Db, hipStream_t st) {
  if (g.dim == 1) { micro_t<1, T, 64, 1>(g, binfo, nslot, lds, dt, crec, h, b, Sh, Sb, Dh, Db, st); return; }
  switch (KC * 4 + R) {
    case 16 * 4 + 1: micro_t<2, T, 16, 1>(g, binfo, nslot, lds, dt, crec, h, b, Sh, Sb, Dh, Db, st); break;
    case 16 * 4 + 2: micro_t<2, T, 16, 2>(g, binfo, nslot, lds, dt, crec, h, b, Sh, Sb, Dh, Db, st); break;
    case 8 * 4 + 1: micro_t<2, T, 8, 1>(g, binfo, nslot, lds, dt, crec, h, b, Sh, Sb, Dh, Db, st); break;
    case 8 * 4 + 2: micro_t<2, T, 8, 2>(g, binfo, nslot, lds, dt, crec, h, b, Sh, Sb, Dh, Db, st); break;
    case 4 * 4 + 1: micro_t<2, T, 4, 1>(g, binfo, nslot, lds, dt, crec, h, b, Sh, Sb, Dh, Db, st); break;
    case 4 * 4 + 2: micro_t<2, T, 4, 2>(g, binfo, nslot, lds, dt, crec, h, b, Sh, Sb, Dh, Db, st); break;
    case 2 * 4 + 1: micro_t<2, T, 2, 1>(g, binfo, nslot, lds, dt, crec, h, b, Sh, Sb, Dh, Db, st); break;
    default: micro_t<2, T, 2, 2>(g, binfo, nslot, lds, dt, crec, h, b, Sh, Sb, Dh, Db, st); break;
  }
}

void launch_micro(const Dev& g, int prec, const int* binfo, int max_ni, int max_nj, int any_pj, double dt,
                  const double* crec, void* h, void* b, const void* Sh, const void* Sb, void* Dh, void* Db,
                  hipStream_t st, hipEvent_t* ev) {
  int KC, R;
  micro_shape(g.dim, max_ni, max_nj, any_pj, g.kc_max, KC, R);
  // the residual pass, unless the forward sweep of this shape forms it
  if (!micro_fused(KC, R)) {
    if (prec == 0)
      k_micro_rhs<double><<<nb4(g.ncell), 256, 0, st>>>(g, dt, crec, (const double*)h, (const double*)b,
                                                        (const double*)Sh, (const double*)Sb, (double*)Dh,
                                                        (double*)Db);
    else
      k_micro_rhs<float><<<nb4(g.ncell), 256, 0, st>>>(g, dt, crec, (const float*)h, (const float*)b,
                                                       (const float*)Sh, (const float*)Sb, (float*)Dh, (float*)Db);
  }
  if (ev) (void)hipEventRecord(ev[0], st);
  const int nslot = (g.dim == 1) ? 1 : max_nj;
  const size_t lds = micro_lds_of(g.dim, max_ni, max_nj, any_pj, KC, R);
  if (prec == 0) micro_prec<double>(g, binfo, KC, R, nslot, lds, dt, crec, Sh, Sb, h, b, Dh, Db, st);
  else micro_prec<float>(g, binfo, KC, R, nslot, lds, dt, crec, Sh, Sb, h, b, Dh, Db, st);
}

// ------------------------------------------------------------------------
// batched pseudo-iteration (BatchPlan): one launch per stage for all cases
// ------------------------------------------------------------------------
// case of flat workgroup `bid`: off[c] <= bid < off[c + 1] (binary search
// over the prefix table; wave-uniform, so scalar loads)
__device__ __forceinline__ int case_of(const int* __restrict__ off, int ncase, int bid) {
  typedef const int __attribute__((address_space(4))) CInt;
  const CInt* o = (const CInt*)off;
  int lo = 0, hi = ncase;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (o[mid] <= bid) lo = mid; else hi = mid;
  }
  return __builtin_amdgcn_readfirstlane(lo);
}

// the case table is read through the constant address space: read-only
// for the whole launch, so its loads are scalar and free to repeat, as for a
// per-case kernel's own argument block
typedef const BatchCase __attribute__((address_space(4))) ConstCase;
__device__ __forceinline__ const BatchCase& const_case(const BatchCase* cs, int i) {
  return *(const BatchCase*)&((ConstCase*)cs)[__builtin_amdgcn_readfirstlane(i)];
}
// a work item (wave-uniform), read through the constant address space
__device__ __forceinline__ BatchItem const_item(const BatchItem* items, int it) {
  typedef const int __attribute__((address_space(4))) CInt;
  const CInt* p = (const CInt*)(items + __builtin_amdgcn_readfirstlane(it));
  return BatchItem{__builtin_amdgcn_readfirstlane(p[0]), __builtin_amdgcn_readfirstlane(p[1]),
                   __builtin_amdgcn_readfirstlane(p[2]), __builtin_amdgcn_readfirstlane(p[3])};
}

#define UGKS_BATCH_CASE(off)                                   \
  const int bc_ = case_of(off, ncase, (int)blockIdx.x);         \
  const BatchCase& a = const_case(cs, bc_);                     \
  const int bx = (int)blockIdx.x - ((const int __attribute__((address_space(4)))*)off)[bc_];

__global__ void kb_gradW(const BatchCase* __restrict__ cs, const int* __restrict__ off, int ncase) {
  UGKS_BATCH_CASE(off)
  gradW_body(bx, a.g, a.W, a.gW);
}
__global__ void kb_wallprep(const BatchCase* __restrict__ cs, const int* __restrict__ off, int ncase) {
  UGKS_BATCH_CASE(off)
  wallprep_body(bx, a.g, a.dts, a.W, a.q, a.gW, a.rec);
}
__global__ void kb_face_fin(const BatchCase* __restrict__ cs, const int* __restrict__ off, int ncase) {
  UGKS_BATCH_CASE(off)
  face_fin_body(bx, a.g, a.dts, a.nchunk, a.part, a.W, a.gW, a.rec);
}
__global__ void kb_flux_fin(const BatchCase* __restrict__ cs, const int* __restrict__ off, int ncase) {
  UGKS_BATCH_CASE(off)
  flux_fin_body(bx, a.g, a.nchunk, a.part, a.rec, a.F, nullptr);
}
__global__ void kb_gamma(const BatchCase* __restrict__ cs, const int* __restrict__ off, int ncase) {
  UGKS_BATCH_CASE(off)
  gamma_body(bx, a.g, a.W, a.gam);
}
__global__ void kb_macro_prep(const BatchCase* __restrict__ cs, const int* __restrict__ off, int ncase) {
  UGKS_BATCH_CASE(off)
  macro_prep_body(bx, a.g, a.dt, a.W, a.Wn, a.F, a.Fn, a.gam, a.mac);
}
__global__ void kb_cellrec(const BatchCase* __restrict__ cs, const int* __restrict__ off, int ncase) {
  UGKS_BATCH_CASE(off)
  cellrec_body(bx, a.g, a.dt, a.Wp, nullptr, a.mrec, a.crec);
}
template <class T>
__global__ __launch_bounds__(256) void kb_interp(const BatchCase* __restrict__ cs, const int* __restrict__ off,
                                                 int ncase) {
  UGKS_BATCH_CASE(off)
  interp_body<T>(bx, a.g, a.nrec, a.orec, a.optr, a.odon, a.ow, (T*)a.h, (T*)a.b, a.W, a.q);
}
template <class T>
__global__ __launch_bounds__(256) void kb_step7(const BatchCase* __restrict__ cs, const int* __restrict__ off,
                                                int ncase, int mode) {
  UGKS_BATCH_CASE(off)
  step7_body<T>(bx, a.g, mode, (const T*)a.h, (const T*)a.b, mode ? a.crec : nullptr, mode ? a.Wp : nullptr, a.W,
                a.q, a.mrec);
}
template <class T>
__global__ __launch_bounds__(256) void kb_micro_rhs(const BatchCase* __restrict__ cs, const int* __restrict__ off,
                                                    int ncase) {
  UGKS_BATCH_CASE(off)
  micro_rhs_body<T>(bx, a.g, a.dt, a.crec, (const T*)a.h, (const T*)a.b, (const T*)a.Sh, (const T*)a.Sb,
                    (T*)a.Dh, (T*)a.Db);
}
template <int NTB>
__global__ __launch_bounds__(NTB) void kb_macro_sweep(const BatchCase* __restrict__ cs, const int* __restrict__ off,
                                                      int ncase, int max_ni, int max_nj, int any_pi, int any_pj) {
  UGKS_BATCH_CASE(off)
  macro_sweep_body<2, NTB>(bx, a.g, a.binfo, a.W, a.mac, a.dWs, a.dW, a.Wp, a.rpart, max_ni, max_nj, any_pi,
                           any_pj);
}
// residual norms of inner iteration s: one workgroup per case
__global__ void kb_resid(const BatchCase* __restrict__ cs, int s) {
  const BatchCase& a = const_case(cs, blockIdx.x);
  if (a.resid) resid_body(a.g.nblock, a.g.nw, a.rpart, a.resid + (size_t)s * a.g.nw);
}
// persistent march: each workgroup takes every gridDim.x-th work item
template <int RG, class T, int MODE>
__global__ __launch_bounds__(64 * (RG + 2)) void kb_march(const BatchCase* __restrict__ cs,
                                                          const BatchItem* __restrict__ items, int nitems) {
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const BatchItem w = const_item(items, it);
    const BatchCase& a = const_case(cs, w.cs);
    march_body<RG, T, T, MODE>(w.x, w.y, w.z, a.g, (cint*)a.binfo, a.nchunk, (const T*)a.h, (const T*)a.b,
                               (cdouble*)a.rec, (cdouble*)a.g.fplan, a.part, (T*)a.Dh, (T*)a.Db);
    __syncthreads();  // the next item reuses the LDS
  }
}
// persistent micro sweep (no chunk-to-XCD remapping: the items are dealt
// round robin already)
template <class T, int KC, int P, int R>
__global__ __launch_bounds__(1024) void kb_micro(const BatchCase* __restrict__ cs,
                                                 const BatchItem* __restrict__ items, int nitems, int nslot) {
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const BatchItem w = const_item(items, it);
    const BatchCase& a = const_case(cs, w.cs);
    micro_body<2, T, KC, P, R>(w.x, 0, w.y, a.g, a.binfo, nslot, a.crec, (T*)a.h, (T*)a.b, (T*)a.Dh, (T*)a.Db,
                               (const T*)a.Sh, (const T*)a.Sb, a.dt);
    __syncthreads();
  }
}
#undef UGKS_BATCH_CASE

template <class T, int KC, int R>
static const void* kb_micro_fn() {
  return (const void*)kb_micro<T, KC, micro_depth<T, KC, R>(), R>;
}
template <class T>
static const void* kb_micro_sel(int KC, int R) {
  switch (KC * 4 + R) {
    case 16 * 4 + 1: return kb_micro_fn<T, 16, 1>();
    case 16 * 4 + 2: return kb_micro_fn<T, 16, 2>();
    case 8 * 4 + 1: return kb_micro_fn<T, 8, 1>();
    case 8 * 4 + 2: return kb_micro_fn<T, 8, 2>();
    case 4 * 4 + 1: return kb_micro_fn<T, 4, 1>();
    case 4 * 4 + 2: return kb_micro_fn<T, 4, 2>();
    case 2 * 4 + 1: return kb_micro_fn<T, 2, 1>();
    default: return kb_micro_fn<T, 2, 2>();
  }
}
template <class T>
static const void* kb_march_sel(int rg, int mode) {
  if (rg == 6) return mode ? (const void*)kb_march<6, T, 1> : (const void*)kb_march<6, T, 0>;
  if (rg == 10) return mode ? (const void*)kb_march<10, T, 1> : (const void*)kb_march<10, T, 0>;
  return mode ? (const void*)kb_march<8, T, 1> : (const void*)kb_march<8, T, 0>;
}

static int micro_threads(int nslot, int KC, int R) { return ((((nslot + R - 1) / R) * KC + 63) / 64) * 64; }

static int cu_count(int& ncu) {
  int dev = 0;
  return (hipGetDevice(&dev) != hipSuccess ||
          hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
             ? -1
             : 0;
}

int batch_march_grid(int prec, int rg, int mode, int& grid) {
  int ncu = 0, a = 0;
  if (cu_count(ncu)) return -1;
  const void* fm = prec ? kb_march_sel<float>(rg, mode) : kb_march_sel<double>(rg, mode);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, fm, 64 * (rg + 2), 0) != hipSuccess) return -1;
  grid = ncu * (a > 0 ? a : 1);
  return 0;
}

int batch_micro_grid(size_t micro_lds, int& grid) {
  int ncu = 0;
  if (cu_count(ncu)) return -1;
  // the sweep's occupancy follows from its LDS (one workgroup holds the
  // hand-off and record slots of its block), at most two 1024-thread
  // workgroups per CU
  const int m = (int)((160 * 1024) / (micro_lds > 0 ? micro_lds : 1));
  grid = ncu * (m > 0 ? (m < 2 ? m : 2) : 1);
  return 0;
}

template <class T>
static void batch_inner_t(const BatchPlan& p, int n_inner, hipStream_t st) {
  const BatchCase* cs = p.cases;
  const int nc = p.ncase;
  kb_step7<T><<<p.n_cell4, 256, 0, st>>>(cs, p.off_cell4, nc, 0);
  const int KC = p.micro_kc, R = p.micro_rows;
  const int mthreads = micro_threads(p.micro_nslot, KC, R);
  for (int s = 0; s < n_inner; ++s) {
    if (p.n_rec4 > 0) kb_interp<T><<<p.n_rec4, 256, 0, st>>>(cs, p.off_rec4, nc);
    kb_gradW<<<p.n_cell64, 64, 0, st>>>(cs, p.off_cell64, nc);
    kb_wallprep<<<p.n_face64, 64, 0, st>>>(cs, p.off_face64, nc);
    for (int mode = 0; mode < 2; ++mode) {
      const int rg = p.rg[mode], gm = p.grid_march[mode], nm = p.n_march[mode];
      const BatchItem* it = p.march_items[mode];
      if (rg == 6) {
        if (mode) kb_march<6, T, 1><<<gm, 64 * 8, 0, st>>>(cs, it, nm);
        else kb_march<6, T, 0><<<gm, 64 * 8, 0, st>>>(cs, it, nm);
      } else if (rg == 10) {
        if (mode) kb_march<10, T, 1><<<gm, 64 * 12, 0, st>>>(cs, it, nm);
        else kb_march<10, T, 0><<<gm, 64 * 12, 0, st>>>(cs, it, nm);
      } else {
        if (mode) kb_march<8, T, 1><<<gm, 64 * 10, 0, st>>>(cs, it, nm);
        else kb_march<8, T, 0><<<gm, 64 * 10, 0, st>>>(cs, it, nm);
      }
      if (mode == 0) kb_face_fin<<<p.n_face64, 64, 0, st>>>(cs, p.off_face64, nc);
    }
    kb_flux_fin<<<p.n_face64, 64, 0, st>>>(cs, p.off_face64, nc);
    kb_gamma<<<p.n_face64, 64, 0, st>>>(cs, p.off_face64, nc);
    kb_macro_prep<<<p.n_cell64, 64, 0, st>>>(cs, p.off_cell64, nc);
    if (p.macro_nt == 64)
      kb_macro_sweep<64><<<p.n_block, 64, p.macro_lds, st>>>(cs, p.off_block, nc, p.max_ni, p.max_nj, p.any_pi,
                                                            p.any_pj);
    else
      kb_macro_sweep<512><<<p.n_block, p.macro_nt, p.macro_lds, st>>>(cs, p.off_block, nc, p.max_ni, p.max_nj,
                                                                      p.any_pi, p.any_pj);
    if (p.want_resid) kb_resid<<<nc, 64, 0, st>>>(cs, s);
    kb_cellrec<<<p.n_cell64, 64, 0, st>>>(cs, p.off_cell64, nc);
    if (!micro_fused(KC, R)) kb_micro_rhs<T><<<p.n_cell4, 256, 0, st>>>(cs, p.off_cell4, nc);
    const void* fn = kb_micro_sel<T>(KC, R);
    const BatchItem* mi = p.micro_items;
    int nmi = p.n_micro, nslot = p.micro_nslot;
    void* args[] = {(void*)&cs, (void*)&mi, (void*)&nmi, (void*)&nslot};
    (void)hipLaunchKernel(fn, dim3((unsigned)p.grid_micro), dim3((unsigned)mthreads), args, p.micro_lds, st);
    kb_step7<T><<<p.n_cell4, 256, 0, st>>>(cs, p.off_cell4, nc, 1);
  }
}

void launch_batch_inner(const BatchPlan& p, int n_inner, hipStream_t st) {
  if (p.prec == 0) batch_inner_t<double>(p, n_inner, st);
  else batch_inner_t<float>(p, n_inner, st);
}

// dynamic LDS limits of the sweep kernels, set once per device before any
// launch (kernel attributes are not stream work, so a captured graph never
// depends on them)
template <class T>
static int micro_attrs() {
  const void* f[] = {(const void*)k_micro<1, T, 64, micro_depth<T, 64, 1>(), 1>,
                     (const void*)k_micro<2, T, 16, micro_depth<T, 16, 1>(), 1>,
                     (const void*)k_micro<2, T, 16, micro_depth<T, 16, 2>(), 2>,
                     (const void*)k_micro<2, T, 8, micro_depth<T, 8, 1>(), 1>,
                     (const void*)k_micro<2, T, 8, micro_depth<T, 8, 2>(), 2>,
                     (const void*)k_micro<2, T, 4, micro_depth<T, 4, 1>(), 1>,
                     (const void*)k_micro<2, T, 4, micro_depth<T, 4, 2>(), 2>,
                     (const void*)k_micro<2, T, 2, micro_depth<T, 2, 1>(), 1>,
                     (const void*)k_micro<2, T, 2, micro_depth<T, 2, 2>(), 2>};
  for (const void* k : f)
    if (hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024) != hipSuccess) return -1;
  return 0;
}

int init_kernel_attributes() {
  if (micro_attrs<double>() || micro_attrs<float>()) return -1;
  for (const void* k : {(const void*)k_macro_sweep<1, 64>, (const void*)k_macro_sweep<2, 64>,
                        (const void*)k_macro_sweep<2, 512>, (const void*)kb_macro_sweep<64>,
                        (const void*)kb_macro_sweep<512>})
    if (hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024) != hipSuccess) return -1;
  for (int kc : {16, 8, 4, 2})
    for (int r : {1, 2})
      for (const void* k : {kb_micro_sel<double>(kc, r), kb_micro_sel<float>(kc, r)})
        if (hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024) != hipSuccess) return -1;
  return 0;
}

}  // namespace ugks

namespace ugks {

// ------------------------------------------------------------------------
// wall loads (Sec. 2.1: the macro flux into an isothermal wall gives the
// pressure and shear load and the heat flux on the body).  The wall table
// lists the wall faces of each (block, side) in face order; entry e holds
// kWt* fields: face id, area, the sign that turns the face normal into the
// normal pointing into the wall, that inward normal, and the face centre
// relative to the block's moved rotation centre.  One thread per (block,
// side) walks its faces in order, so the sums are reproducible.
// ------------------------------------------------------------------------
__global__ void k_fill(double* __restrict__ a, size_t n, double v) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

__global__ void k_wall_loads(Dev g, int nside, const int* __restrict__ wptr, const double* __restrict__ wtab,
                             const double* __restrict__ F, double* __restrict__ face_out,
                             double* __restrict__ side_out) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nside) return;
  const int D = g.dim, nw = g.nw;
  double fx = 0.0, fy = 0.0, mz = 0.0, qe = 0.0;
  for (int e = wptr[s]; e < wptr[s + 1]; ++e) {
    const double* t = wtab + (size_t)e * kWtN;
    const int f = tab_int(t[kWtFace]);
    const double S = t[kWtS], sg = t[kWtSgn], nix = t[kWtNx], niy = t[kWtNy];
    const double* Ff = F + (size_t)f * nw;
    // flux into the wall per unit area: momentum (the load on the body)
    // and energy
    const double mx = sg * Ff[1], my = (D == 2) ? sg * Ff[2] : 0.0, en = sg * Ff[D + 1];
    if (face_out) {
      double* o = face_out + (size_t)f * (D + 3);
      o[0] = mx;
      if (D == 2) o[1] = my;
      o[D] = mx * nix + my * niy;        // pressure load p_w
      o[D + 1] = -mx * niy + my * nix;   // shear load sigma_w along (-n_y, n_x)
      o[D + 2] = en;                     // heat flux q_w
    }
    fx += S * mx;
    fy += S * my;
    mz += S * (t[kWtRx] * my - t[kWtRy] * mx);
    qe += S * en;
  }
  if (side_out) {
    double* o = side_out + (size_t)s * 4;
    o[0] = fx; o[1] = fy; o[2] = mz; o[3] = qe;
  }
}

// transpose of k_wall_loads with respect to F (F_bar of non-wall faces is
// zeroed before)
__global__ void k_wall_loads_adj(Dev g, int nside, const int* __restrict__ wptr, const double* __restrict__ wtab,
                                 const double* __restrict__ face_bar, const double* __restrict__ side_bar,
                                 double* __restrict__ F_bar) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nside) return;
  const int D = g.dim, nw = g.nw;
  const double* sb = side_bar ? side_bar + (size_t)s * 4 : nullptr;
  for (int e = wptr[s]; e < wptr[s + 1]; ++e) {
    const double* t = wtab + (size_t)e * kWtN;
    const int f = tab_int(t[kWtFace]);
    const double S = t[kWtS], sg = t[kWtSgn], nix = t[kWtNx], niy = t[kWtNy];
    double bmx = 0.0, bmy = 0.0, ben = 0.0;
    if (face_bar) {
      const double* o = face_bar + (size_t)f * (D + 3);
      bmx = o[0] + o[D] * nix - o[D + 1] * niy;
      if (D == 2) bmy = o[1] + o[D] * niy + o[D + 1] * nix;
      ben = o[D + 2];
    }
    if (sb) {
      bmx += S * (sb[0] - t[kWtRy] * sb[2]);
      bmy += S * (sb[1] + t[kWtRx] * sb[2]);
      ben += S * sb[3];
    }
    double* Fb = F_bar + (size_t)f * nw;
    Fb[1] = sg * bmx;
    if (D == 2) Fb[2] = sg * bmy;
    Fb[D + 1] = sg * ben;
  }
}

// rigid-velocity and wall-RT cotangents of each block from the per-face
// cotangents [nface][5] (face grid velocity x, y; wall velocity x, y; wall
// RT): one workgroup of 256 threads per block sums its faces (strided, then
// a fixed tree), and four threads sum the wall RT entries of its sides
__global__ __launch_bounds__(256) void k_param_bars(int nblock, const int* __restrict__ bface,
                                                    const int* __restrict__ wptr, const double* __restrict__ wtab,
                                                    const double* __restrict__ face_bar, double* __restrict__ U_bar,
                                                    double* __restrict__ rtw_bar) {
  __shared__ double red[2][256];
  const int b = blockIdx.x, t = threadIdx.x;
  if (b >= nblock) return;
  double sx = 0.0, sy = 0.0;
  for (int f = bface[b] + t; f < bface[b + 1]; f += 256) {
    const double* fb = face_bar + (size_t)f * 5;
    sx += fb[0] + fb[2];
    sy += fb[1] + fb[3];
  }
  red[0][t] = sx;
  red[1][t] = sy;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) { red[0][t] += red[0][t + w]; red[1][t] += red[1][t + w]; }
    __syncthreads();
  }
  if (t == 0) { U_bar[2 * b] = red[0][0]; U_bar[2 * b + 1] = red[1][0]; }
  if (t < 4) {
    const int s = 4 * b + t;
    double r = 0.0;
    for (int e = wptr[s]; e < wptr[s + 1]; ++e) r += face_bar[(size_t)tab_int(wtab[(size_t)e * kWtN + kWtFace]) * 5 + 4];
    rtw_bar[s] = r;
  }
}

void launch_fill(double* a, size_t n, double v, hipStream_t st) {
  if (n > 0) k_fill<<<nbl(n, 256), 256, 0, st>>>(a, n, v);
}

void launch_wall_loads(const Dev& g, int nside, const int* wptr, const double* wtab, const double* F,
                       double* face_out, double* side_out, hipStream_t st) {
  if (face_out) launch_fill(face_out, (size_t)g.nface * (g.dim + 3), 0.0, st);
  k_wall_loads<<<nbl(nside, 64), 64, 0, st>>>(g, nside, wptr, wtab, F, face_out, side_out);
}

void launch_wall_loads_adj(const Dev& g, int nside, const int* wptr, const double* wtab, const double* face_bar,
                           const double* side_bar, double* F_bar, hipStream_t st) {
  launch_fill(F_bar, (size_t)g.nface * g.nw, 0.0, st);
  k_wall_loads_adj<<<nbl(nside, 64), 64, 0, st>>>(g, nside, wptr, wtab, face_bar, side_bar, F_bar);
}

void launch_param_bars(int nblock, const int* bface, const int* wptr, const double* wtab, const double* face_bar,
                       double* U_bar, double* rtw_bar, hipStream_t st) {
  k_param_bars<<<nblock, 256, 0, st>>>(nblock, bface, wptr, wtab, face_bar, U_bar, rtw_bar);
}

}  // namespace ugks

// ------------------------------------------------------------------------
// scratch of the entry points that allocate nothing: one file-scope device
// array, each device holding its own copy (at its own address) while the
// process lives.  Its host-side name is not a device address: the address
// is looked up once per device, with that device current, and cached.
// ------------------------------------------------------------------------
namespace {
static __device__ __align__(256) char scratch[ugks::kStaticScratchBytes];
std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;  // per device
}  // namespace

namespace ugks {

int static_scratch(int device, void** ptr) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (device < 0) return -1;
  if ((int)g_scratch_ptr.size() <= device) g_scratch_ptr.resize(device + 1, nullptr);
  if (!g_scratch_ptr[device]) {
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return -1;
    if (cur != device && hipSetDevice(device) != hipSuccess) return -1;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess || !p) return -1;
    g_scratch_ptr[device] = p;
  }
  *ptr = g_scratch_ptr[device];
  return 0;
}

}  // namespace ugks
