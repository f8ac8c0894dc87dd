// libugks host side: the C ABI of include/ugks.h, problem setup, host
// geometry of the moving structured blocks and the pseudo-iteration driver.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "ugks.h"
#include "ugks_adjoint.h"
#include "ugks_kernels.h"
#include "ugks_overset.h"

using namespace ugks;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIPCHK(x)                                                                      \
  do {                                                                                 \
    hipError_t e_ = (x);                                                               \
    if (e_ != hipSuccess) return fail(UGKS_E_DEVICE, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

struct Block {
  int ni, nj, bc[4];
  double rtw[4], vwx[4], vwy[4], xc0, yc0;
  std::vector<double> x0, y0;  // reference nodes
  double pose[6] = {0, 0, 0, 0, 0, 0};
  int cell0, face_i0, face_j0;
};

template <class T>
struct DBuf {
  T* p = nullptr;
  size_t n = 0;
};

}  // namespace

struct ugks_ctx {
  int device = 0;
  // captured pseudo-iterations: the graph is rebuilt when its key changes;
  // `version` counts changes of geometry, cell kinds and donor tables
  unsigned version = 0;
  hipStream_t cap = nullptr;
  hipGraphExec_t gexec = nullptr;
  std::vector<uint64_t> gkey;
  int dim = 2, nxi = 1, nw = 4, prec = 0;
  double pr, omega, mu_ref, rt_ref, cfl_s, cfl_p;
  int nvx, nvy, nv;
  double vrange[4];
  double winf[4] = {0, 0, 0, 0};
  std::vector<double> vx, vy, wk;  // per k
  std::vector<Block> blk;
  int ncell = 0, nface = 0;
  int max_ni = 0, max_nj = 0, any_pi = 0, any_pj = 0;
  // host geometry
  std::vector<double> xn, yn;  // current nodes, per block
  std::vector<size_t> node0;
  std::vector<double> vol, G, cdx, dtp, fgeo, mgeo, ccx, ccy;  // ccx, ccy: cell centroids
  std::vector<double> cplan, fplan;                            // packed march tables
  std::vector<int> nb, cf, fcell;
  std::vector<int8_t> type, fact;
  std::vector<int> cblk, ci, cj;
  double dts = 0.0;
  // device copies
  Dev dev{};
  void *d_vx = nullptr, *d_vy = nullptr, *d_wk = nullptr, *d_vol = nullptr, *d_G = nullptr, *d_cdx = nullptr,
       *d_dtp = nullptr, *d_type = nullptr, *d_nb = nullptr, *d_cf = nullptr, *d_fcell = nullptr,
       *d_fgeo = nullptr, *d_fact = nullptr, *d_cplan = nullptr, *d_fplan = nullptr, *d_finf_h = nullptr, *d_finf_b = nullptr, *d_binfo = nullptr,
       *d_mgeo = nullptr;
  // scratch
  void *s_gW = nullptr, *s_rec = nullptr, *s_gam = nullptr, *s_R = nullptr, *s_Dg = nullptr, *s_dWs = nullptr,
       *s_dW = nullptr, *s_Wp = nullptr, *s_rpart = nullptr, *s_crec = nullptr, *s_mrec = nullptr,
       *s_Dh = nullptr, *s_Db = nullptr, *s_F = nullptr, *s_part = nullptr;
  // overset
  int nrec = 0;  // receptor rows of the donor table
  int nref = 0;  // rows after them: cells uncovered from holes, interpolated once
  void *d_rec = nullptr, *d_ptr = nullptr, *d_don = nullptr, *d_w = nullptr;
  std::vector<int> h_rec, h_ptr, h_don;
  std::vector<double> h_w;
  // workspace of the reverse-mode entry points (allocated on first use, or
  // carved from a caller's workspace)
  std::vector<void*> adj;
  // write-disjoint colourings of the reverse-mode scatters: faces other than
  // wall faces, cells, receptor rows, refill rows, wall faces (items in that
  // order in the workspace buffer A_ORD, colour offsets on the host), for
  // the tables of version `ord_version`
  long long ord_version = -1;
  std::vector<int> ord_off[5];
  // scratch: one block, owned (allocated at creation) or the caller's
  void* scratch = nullptr;
  bool own_scratch = true;
  bool own_adj = true;
  // device status word (kStatus* bits) and the synchronising check mode
  unsigned* d_status = nullptr;
  int sync_check = 0;
  // wall table (kWt* entries per wall face, grouped by block side) and the
  // face range of each block
  std::vector<double> wtab;
  std::vector<int> wptr, bface;
  void *d_wtab = nullptr, *d_wptr = nullptr, *d_bface = nullptr;
  void* d_side = nullptr;  // [nblock][4][4] side loads of the body motion
  // this device's address of the library's static scratch array (entry
  // points that allocate nothing), looked up at creation; null if the
  // lookup failed
  void* sscratch = nullptr;
};

namespace {


// composite closed Newton-Cotes weights on n uniform points of [a, b]
// (Boole if (n-1) % 4 == 0; Simpson for odd n; Simpson | 3/8 | Simpson for
// n % 4 == 0; Simpson | 3/8 | 3/8 | 3/8 | Simpson for n % 4 == 2, n >= 10)
std::vector<double> nc_weights(int n, double a, double b) {
  std::vector<double> w(n, 0.0);
  if (n == 1) { w[0] = 1.0; return w; }
  double h = (b - a) / (n - 1);
  if (n == 2) { w[0] = w[1] = 0.5 * h; return w; }
  auto simpson = [&](int i0, int m) {
    for (int p = i0; p < i0 + m; p += 2) { w[p] += h / 3.0; w[p + 1] += 4.0 * h / 3.0; w[p + 2] += h / 3.0; }
  };
  auto three8 = [&](int i0) {
    w[i0] += 3.0 * h / 8.0; w[i0 + 1] += 9.0 * h / 8.0; w[i0 + 2] += 9.0 * h / 8.0; w[i0 + 3] += 3.0 * h / 8.0;
  };
  int m = n - 1;
  if (m % 4 == 0) {
    for (int p = 0; p < m; p += 4) {
      w[p] += 14.0 * h / 45.0; w[p + 1] += 64.0 * h / 45.0; w[p + 2] += 24.0 * h / 45.0;
      w[p + 3] += 64.0 * h / 45.0; w[p + 4] += 14.0 * h / 45.0;
    }
  } else if (n % 2 == 1) {
    simpson(0, m);
  } else if (n % 4 == 0) {
    int s = (n - 4) / 2;
    simpson(0, s); three8(s); simpson(s + 3, s);
  } else if (n >= 10) {
    int s = (n - 4) / 2 - 3;
    simpson(0, s); three8(s); three8(s + 3); three8(s + 6); simpson(s + 9, s);
  } else {
    simpson(0, n - 4); three8(n - 4);
  }
  return w;
}

template <class T>
int upload(void*& d, const std::vector<T>& h) {
  size_t bytes = std::max<size_t>(1, h.size()) * sizeof(T);
  if (!d) HIPCHK(hipMalloc(&d, bytes));
  if (!h.empty()) HIPCHK(hipMemcpy(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
  return UGKS_OK;
}

int alloc(void*& d, size_t bytes) {
  if (d) return UGKS_OK;
  HIPCHK(hipMalloc(&d, std::max<size_t>(bytes, 256)));
  return UGKS_OK;
}

void prim(const ugks_ctx* c, const double* W, double& rho, double& ux, double& uy, double& lam) {
  rho = W[0];
  ux = W[1] / rho;
  uy = (c->dim == 2) ? W[2] / rho : 0.0;
  double e = W[c->dim + 1] - 0.5 * rho * (ux * ux + uy * uy);
  lam = 0.25 * (double)(c->dim + c->nxi) * rho / e;
}

int cell_of(const ugks_ctx* c, int b, int i, int j) { return c->blk[b].cell0 + i + c->blk[b].ni * j; }

// neighbour code of cell (b, i, j) in slot s
int neighbour(const ugks_ctx* c, int cell, int s) {
  int b = c->cblk[cell], i = c->ci[cell], j = c->cj[cell];
  const Block& B = c->blk[b];
  int dir = s / 2, side = (s & 1) ? 1 : -1;
  if (c->dim == 1 && dir == 1) return kNbMiss;
  int ii = i + (dir == 0 ? side : 0), jj = j + (dir == 1 ? side : 0);
  int n = (dir == 0) ? B.ni : B.nj;
  int idx = (dir == 0) ? ii : jj;
  if (idx < 0 || idx >= n) {
    if (B.bc[2 * dir] == UGKS_BC_PERIODIC) {
      idx = (idx + n) % n;
      if (dir == 0) ii = idx; else jj = idx;
    } else {
      switch (B.bc[s]) {
        case UGKS_BC_FARFIELD: return kNbFar;
        case UGKS_BC_COPY: return kNbCopy;
        case UGKS_BC_WALL: return kNbWall;
        default: return kNbMiss;
      }
    }
  }
  int o = cell_of(c, b, ii, jj);
  return c->type[o] == UGKS_HOLE ? kNbMiss : o;
}

// topology tables that depend on the cell kinds
void build_tables(ugks_ctx* c) {
  c->nb.assign(4 * (size_t)c->ncell, kNbMiss);
  for (int n = 0; n < c->ncell; ++n)
    for (int s = 0; s < 4; ++s) c->nb[4 * n + s] = neighbour(c, n, s);
  c->fact.assign(c->nface, 0);
  for (int f = 0; f < c->nface; ++f) {
    int L = c->fcell[2 * f], R = c->fcell[2 * f + 1];
    bool a = (L >= 0 && c->type[L] == UGKS_FIELD) || (R >= 0 && c->type[R] == UGKS_FIELD);
    bool valid = !(L == kNbMiss || R == kNbMiss);
    c->fact[f] = (a && valid) ? 1 : 0;
  }
}

// face numbering and the static face-cell table
void build_faces(ugks_ctx* c) {
  int nf = 0;
  for (auto& B : c->blk) {
    B.face_i0 = nf;
    nf += (B.ni + 1) * B.nj;
    B.face_j0 = nf;
    if (c->dim == 2) nf += B.ni * (B.nj + 1);
  }
  c->nface = nf;
  c->fcell.assign(2 * (size_t)nf, kNbMiss);
  c->cf.assign(4 * (size_t)c->ncell, -1);
  for (int b = 0; b < (int)c->blk.size(); ++b) {
    const Block& B = c->blk[b];
    for (int dir = 0; dir < c->dim; ++dir) {
      bool per = B.bc[2 * dir] == UGKS_BC_PERIODIC;
      int nI = (dir == 0) ? B.ni + 1 : B.ni, nJ = (dir == 0) ? B.nj : B.nj + 1;
      for (int j = 0; j < nJ; ++j)
        for (int i = 0; i < nI; ++i) {
          int f = (dir == 0) ? B.face_i0 + i + (B.ni + 1) * j : B.face_j0 + i + B.ni * j;
          int idx = (dir == 0) ? i : j, n = (dir == 0) ? B.ni : B.nj;
          if (per && idx == n) continue;  // duplicate of face 0 of the row
          int L, R;
          int lo_cell = (idx > 0) ? cell_of(c, b, dir == 0 ? i - 1 : i, dir == 0 ? j : j - 1)
                                  : (per ? cell_of(c, b, dir == 0 ? n - 1 : i, dir == 0 ? j : n - 1) : -1);
          int hi_cell = (idx < n) ? cell_of(c, b, i, j) : -1;
          auto code = [&](int side) -> int {
            switch (B.bc[side]) {
              case UGKS_BC_FARFIELD: return kNbFar;
              case UGKS_BC_COPY: return kNbCopy;
              case UGKS_BC_WALL: return kNbWall;
              default: return kNbMiss;
            }
          };
          L = (lo_cell >= 0) ? lo_cell : code(2 * dir);
          R = (hi_cell >= 0) ? hi_cell : code(2 * dir + 1);
          if (L == kNbMiss || R == kNbMiss) continue;  // fringe side: no face
          c->fcell[2 * f] = L;
          c->fcell[2 * f + 1] = R;
          if (L >= 0) c->cf[4 * L + 2 * dir + 1] = f;
          if (R >= 0) c->cf[4 * R + 2 * dir] = f;
        }
    }
  }
}

// node positions, cell and face geometry, time steps at the current poses
// vertices of the convex hull of the velocity points: the four corners of a
// uniform grid (in the order x-min/max by y-min/max), Andrew's monotone
// chain for an unstructured mesh
static std::vector<std::pair<double, double>> velocity_hull(const ugks_ctx* c) {
  std::vector<std::pair<double, double>> h;
  if (c->nvy > 1 || c->dim == 1) {
    const double vxs[2] = {c->vx[0], c->vx[c->nv - 1]};
    const double vys[2] = {c->vy[0], c->vy[c->nv - 1]};
    for (int a = 0; a < 2; ++a)
      for (int e = 0; e < 2; ++e) h.push_back({vxs[a], vys[e]});
    return h;
  }
  std::vector<std::pair<double, double>> p(c->nv);
  for (int k = 0; k < c->nv; ++k) p[k] = {c->vx[k], c->vy[k]};
  std::sort(p.begin(), p.end());
  p.erase(std::unique(p.begin(), p.end()), p.end());
  if (p.size() < 3) return p;
  auto cross = [](const std::pair<double, double>& o, const std::pair<double, double>& a,
                  const std::pair<double, double>& b) {
    return (a.first - o.first) * (b.second - o.second) - (a.second - o.second) * (b.first - o.first);
  };
  std::vector<std::pair<double, double>> H(2 * p.size());
  size_t k = 0;
  for (size_t i = 0; i < p.size(); ++i) {
    while (k >= 2 && cross(H[k - 2], H[k - 1], p[i]) <= 0) --k;
    H[k++] = p[i];
  }
  for (size_t i = p.size() - 1, t = k + 1; i > 0; --i) {
    while (k >= t && cross(H[k - 2], H[k - 1], p[i - 1]) <= 0) --k;
    H[k++] = p[i - 1];
  }
  H.resize(k - 1);
  return H;
}

void compute_geometry(ugks_ctx* c) {
  int d = c->dim;
  for (int b = 0; b < (int)c->blk.size(); ++b) {
    Block& B = c->blk[b];
    double cs = std::cos(B.pose[2]), sn = std::sin(B.pose[2]);
    size_t nn = B.x0.size();
    for (size_t n = 0; n < nn; ++n) {
      double rx = B.x0[n] - B.xc0, ry = (d == 2) ? B.y0[n] - B.yc0 : 0.0;
      c->xn[c->node0[b] + n] = B.xc0 + B.pose[0] + (cs * rx - sn * ry);
      c->yn[c->node0[b] + n] = (d == 2) ? B.yc0 + B.pose[1] + (sn * rx + cs * ry) : 0.0;
    }
  }
  auto X = [&](int b, int i, int j) { return c->xn[c->node0[b] + i + (size_t)(c->blk[b].ni + 1) * j]; };
  auto Y = [&](int b, int i, int j) { return c->yn[c->node0[b] + i + (size_t)(c->blk[b].ni + 1) * j]; };
  for (int n = 0; n < c->ncell; ++n) {
    int b = c->cblk[n], i = c->ci[n], j = c->cj[n];
    double* G = &c->G[4 * (size_t)n];
    double* D = &c->cdx[8 * (size_t)n];
    if (d == 1) {
      double xa = X(b, i, 0), xb = X(b, i + 1, 0);
      c->vol[n] = xb - xa;
      double xc = 0.5 * (xa + xb);
      c->ccx[n] = xc; c->ccy[n] = 0.0;
      G[0] = 1.0 / (xb - xa); G[1] = G[2] = G[3] = 0.0;
      for (int q = 0; q < 8; ++q) D[q] = 0.0;
      D[0] = xa - xc;
      D[2] = xb - xc;
      continue;
    }
    double px[4] = {X(b, i, j), X(b, i + 1, j), X(b, i + 1, j + 1), X(b, i, j + 1)};
    double py[4] = {Y(b, i, j), Y(b, i + 1, j), Y(b, i + 1, j + 1), Y(b, i, j + 1)};
    double A = 0.0, sx = 0.0, sy = 0.0;
    for (int k = 0; k < 4; ++k) {
      int k1 = (k + 1) % 4;
      double cr = px[k] * py[k1] - px[k1] * py[k];
      A += cr; sx += (px[k] + px[k1]) * cr; sy += (py[k] + py[k1]) * cr;
    }
    A *= 0.5;
    double xc = sx / (6.0 * A), yc = sy / (6.0 * A);
    c->vol[n] = A;
    c->ccx[n] = xc; c->ccy[n] = yc;
    double xxi = 0.5 * (px[1] + px[2]) - 0.5 * (px[0] + px[3]);
    double yxi = 0.5 * (py[1] + py[2]) - 0.5 * (py[0] + py[3]);
    double xet = 0.5 * (px[3] + px[2]) - 0.5 * (px[0] + px[1]);
    double yet = 0.5 * (py[3] + py[2]) - 0.5 * (py[0] + py[1]);
    double det = xxi * yet - xet * yxi;
    G[0] = yet / det; G[1] = -yxi / det; G[2] = -xet / det; G[3] = xxi / det;
    double fx[4] = {0.5 * (px[0] + px[3]), 0.5 * (px[1] + px[2]), 0.5 * (px[0] + px[1]), 0.5 * (px[3] + px[2])};
    double fy[4] = {0.5 * (py[0] + py[3]), 0.5 * (py[1] + py[2]), 0.5 * (py[0] + py[1]), 0.5 * (py[3] + py[2])};
    for (int q = 0; q < 4; ++q) { D[2 * q] = fx[q] - xc; D[2 * q + 1] = fy[q] - yc; }
  }
  // faces; wall faces are listed per block side for the wall loads
  c->fgeo.assign(8 * (size_t)c->nface, 0.0);
  const size_t nside = 4 * c->blk.size();
  std::vector<std::vector<double>> wall_of(nside);
  for (int b = 0; b < (int)c->blk.size(); ++b) {
    const Block& B = c->blk[b];
    double cxm = B.xc0 + B.pose[0], cym = B.yc0 + B.pose[1];
    for (int dir = 0; dir < d; ++dir) {
      int nI = (dir == 0) ? B.ni + 1 : B.ni, nJ = (dir == 0) ? B.nj : B.nj + 1;
      for (int j = 0; j < nJ; ++j)
        for (int i = 0; i < nI; ++i) {
          int f = (dir == 0) ? B.face_i0 + i + (B.ni + 1) * j : B.face_j0 + i + B.ni * j;
          double* g = &c->fgeo[8 * (size_t)f];
          double xf, yf;
          if (d == 1) {
            g[0] = 1.0; g[1] = 0.0; g[2] = 1.0;
            xf = X(b, i, 0); yf = 0.0;
          } else {
            double x0 = X(b, i, j), y0 = Y(b, i, j);
            double x1 = (dir == 0) ? X(b, i, j + 1) : X(b, i + 1, j);
            double y1 = (dir == 0) ? Y(b, i, j + 1) : Y(b, i + 1, j);
            double ex = x1 - x0, ey = y1 - y0;
            double S = std::sqrt(ex * ex + ey * ey);
            g[2] = S;
            if (dir == 0) { g[0] = ey / S; g[1] = -ex / S; }
            else { g[0] = -ey / S; g[1] = ex / S; }
            xf = 0.5 * (x0 + x1); yf = 0.5 * (y0 + y1);
          }
          double rx = xf - cxm, ry = yf - cym;
          g[3] = B.pose[3] - B.pose[5] * ry;
          g[4] = (d == 2) ? B.pose[4] + B.pose[5] * rx : 0.0;
          int L = c->fcell[2 * f], R = c->fcell[2 * f + 1];
          int side = -1;
          if (L == kNbWall) side = 2 * dir;
          if (R == kNbWall) side = 2 * dir + 1;
          if (side >= 0) {
            g[5] = g[3] + B.vwx[side];
            g[6] = (d == 2) ? g[4] + B.vwy[side] : 0.0;
            g[7] = B.rtw[side];
            const double sg = (R == kNbWall) ? 1.0 : -1.0;
            double e[kWtN] = {0.0};
            e[kWtFace] = tab_int_entry(f);
            e[kWtS] = g[2]; e[kWtSgn] = sg; e[kWtNx] = sg * g[0]; e[kWtNy] = sg * g[1];
            e[kWtRx] = rx; e[kWtRy] = ry;
            auto& v = wall_of[4 * (size_t)b + side];
            v.insert(v.end(), e, e + kWtN);
          }
        }
    }
  }
  c->wtab.clear();
  c->wptr.assign(nside + 1, 0);
  for (size_t q = 0; q < nside; ++q) {
    c->wtab.insert(c->wtab.end(), wall_of[q].begin(), wall_of[q].end());
    c->wptr[q + 1] = (int)(c->wtab.size() / kWtN);
  }
  // time steps: max_k |(v_k - U_f).n| (a convex function of v) is reached
  // at a vertex of the velocity points' convex hull: the corners of a
  // uniform grid's box, the hull of an unstructured mesh
  std::vector<double> smax(c->nface, 0.0);
  const std::vector<std::pair<double, double>> hull = velocity_hull(c);
  for (int f = 0; f < c->nface; ++f) {
    const double* g = &c->fgeo[8 * (size_t)f];
    double m = 0.0;
    for (const auto& v : hull) {
      double w = std::fabs((v.first - g[3]) * g[0] + (v.second - g[4]) * g[1]);
      m = std::max(m, w);
    }
    smax[f] = m;
  }
  double dts = INFINITY;
  for (int n = 0; n < c->ncell; ++n) {
    double s = 0.0;
    for (int q = 0; q < 4; ++q) {
      int f = c->cf[4 * (size_t)n + q];
      if (f >= 0) s += 0.5 * c->fgeo[8 * (size_t)f + 2] * smax[f];
    }
    c->dtp[n] = c->cfl_p * c->vol[n] / s;
    if (c->type[n] == UGKS_FIELD) dts = std::min(dts, c->cfl_s * c->vol[n] / s);
  }
  c->dts = dts;
  // micro sweep face coefficients: S/(2|Omega|) (v - U).n_out = A vx + B vy - C
  c->mgeo.assign(12 * (size_t)c->ncell, 0.0);
  for (int n = 0; n < c->ncell; ++n)
    for (int s = 0; s < 4; ++s) {
      int f = c->cf[4 * (size_t)n + s];
      if (f < 0) continue;
      const double* g = &c->fgeo[8 * (size_t)f];
      double sg = (s & 1) ? 1.0 : -1.0;
      double coef = g[2] / (2.0 * c->vol[n]);
      double* m = &c->mgeo[12 * (size_t)n + 3 * s];
      m[0] = coef * sg * g[0];
      m[1] = coef * sg * g[1];
      m[2] = coef * sg * (g[3] * g[0] + g[4] * g[1]);
    }
}

// packed per-cell and per-face tables of the march kernels
int upload_plans(ugks_ctx* c) {
  // built once both the geometry and the topology tables exist
  if (c->vol.size() != (size_t)c->ncell || c->fgeo.size() != 8 * (size_t)c->nface ||
      c->nb.size() != 4 * (size_t)c->ncell || c->cf.size() != 4 * (size_t)c->ncell ||
      c->fact.size() != (size_t)c->nface || c->fcell.size() != 2 * (size_t)c->nface ||
      c->cdx.size() != 8 * (size_t)c->ncell || c->G.size() != 4 * (size_t)c->ncell)
    return UGKS_OK;
  c->cplan.assign((size_t)kCpN * c->ncell, 0.0);
  for (int n = 0; n < c->ncell; ++n) {
    double* P = &c->cplan[(size_t)kCpN * n];
    P[kCpType] = tab_int_entry(c->type[n]);
    for (int s = 0; s < 4; ++s) {
      const int f = c->cf[4 * (size_t)n + s];
      P[kCpNb + s] = tab_int_entry(c->nb[4 * (size_t)n + s]);
      P[kCpG + s] = c->G[4 * (size_t)n + s];
      P[kCpS + s] = (f >= 0) ? c->fgeo[8 * (size_t)f + 2] : 0.0;
      P[kCpFace + s] = tab_int_entry(f);
    }
    P[kCpIvol] = 1.0 / c->vol[n];
  }
  c->fplan.assign((size_t)kFpN * c->nface, 0.0);
  for (int f = 0; f < c->nface; ++f) {
    double* P = &c->fplan[(size_t)kFpN * f];
    const double* fg = &c->fgeo[8 * (size_t)f];
    P[kFpN0] = fg[0]; P[kFpN0 + 1] = fg[1]; P[kFpS] = fg[2]; P[kFpU] = fg[3]; P[kFpU + 1] = fg[4];
    const int L = c->fcell[2 * (size_t)f], R = c->fcell[2 * (size_t)f + 1];
    P[kFpL] = tab_int_entry(L); P[kFpR] = tab_int_entry(R); P[kFpAct] = tab_int_entry(c->fact[f]);
    for (int side = 0; side < 2; ++side) {
      const int cell = side ? R : L;
      if (cell < 0) continue;
      for (int s = 0; s < 4; ++s)
        if (c->cf[4 * (size_t)cell + s] == f) {
          P[(side ? kFpDR : kFpDL)] = c->cdx[8 * (size_t)cell + 2 * s];
          P[(side ? kFpDR : kFpDL) + 1] = c->cdx[8 * (size_t)cell + 2 * s + 1];
        }
    }
  }
  int rc = upload(c->d_cplan, c->cplan);
  if (!rc) rc = upload(c->d_fplan, c->fplan);
  return rc;
}

int upload_geometry(ugks_ctx* c) {
  int rc;
  if ((rc = upload(c->d_vol, c->vol))) return rc;
  if ((rc = upload(c->d_G, c->G))) return rc;
  if ((rc = upload(c->d_cdx, c->cdx))) return rc;
  if ((rc = upload(c->d_dtp, c->dtp))) return rc;
  if ((rc = upload(c->d_fgeo, c->fgeo))) return rc;
  if ((rc = upload(c->d_mgeo, c->mgeo))) return rc;
  if ((rc = upload(c->d_wptr, c->wptr))) return rc;
  if ((rc = upload(c->d_wtab, c->wtab))) return rc;
  return upload_plans(c);
}

int upload_tables(ugks_ctx* c) {
  int rc;
  if ((rc = upload(c->d_type, c->type))) return rc;
  if ((rc = upload(c->d_nb, c->nb))) return rc;
  if ((rc = upload(c->d_fact, c->fact))) return rc;
  return upload_plans(c);
}

void fill_dev(ugks_ctx* c) {
  Dev& g = c->dev;
  g.dim = c->dim; g.nxi = c->nxi; g.nw = c->nw; g.nv = c->nv; g.nvx = c->nvx; g.nvy = c->nvy;
  g.ncell = c->ncell; g.nface = c->nface; g.nblock = (int)c->blk.size();
  g.pr = c->pr; g.omega = c->omega; g.mu_ref = c->mu_ref; g.rt_ref = c->rt_ref;
  for (int m = 0; m < 4; ++m) g.winf[m] = c->winf[m];
  g.vx = (const double*)c->d_vx; g.vy = (const double*)c->d_vy; g.wk = (const double*)c->d_wk;
  g.vol = (const double*)c->d_vol; g.G = (const double*)c->d_G; g.cdx = (const double*)c->d_cdx;
  g.dtp = (const double*)c->d_dtp; g.type = (const int8_t*)c->d_type; g.nb = (const int*)c->d_nb;
  g.cf = (const int*)c->d_cf; g.fcell = (const int*)c->d_fcell; g.fgeo = (const double*)c->d_fgeo;
  g.fact = (const int8_t*)c->d_fact; g.finf_h = c->d_finf_h; g.finf_b = c->d_finf_b;
  g.mgeo = (const double*)c->d_mgeo;
  g.cplan = (const double*)c->d_cplan;
  g.fplan = (const double*)c->d_fplan;
}

// the far-field Maxwellian of c->winf (ghost value of far-field sides) in
// storage precision, to the device
int upload_farfield(ugks_ctx* c) {
  std::vector<double> fh(c->nv), fb(c->nv);
  double rho, ux, uy, lam;
  prim(c, c->winf, rho, ux, uy, lam);
  double nrm = rho * std::pow(lam / kPi, 0.5 * c->dim);
  for (int k = 0; k < c->nv; ++k) {
    double cx = c->vx[k] - ux, cy = (c->dim == 2) ? c->vy[k] - uy : 0.0;
    fh[k] = nrm * std::exp(-lam * (cx * cx + cy * cy));
    fb[k] = (double)c->nxi * 0.5 / lam * fh[k];
  }
  if (c->prec == UGKS_F64) {
    int rc = upload(c->d_finf_h, fh);
    return rc ? rc : upload(c->d_finf_b, fb);
  }
  std::vector<float> a(fh.begin(), fh.end()), e(fb.begin(), fb.end());
  int rc = upload(c->d_finf_h, a);
  return rc ? rc : upload(c->d_finf_b, e);
}

void free_all(ugks_ctx* c) {
  void* ps[] = {c->d_vx, c->d_vy, c->d_wk, c->d_vol, c->d_G, c->d_cdx, c->d_dtp, c->d_type, c->d_nb, c->d_cf,
                c->d_fcell, c->d_fgeo, c->d_fact, c->d_finf_h, c->d_finf_b, c->d_binfo, c->d_mgeo, c->d_rec,
                c->d_ptr, c->d_don, c->d_w, c->d_cplan, c->d_fplan, c->d_status, c->d_wtab, c->d_wptr,
                c->d_bface, c->d_side};
  for (void* p : ps)
    if (p) (void)hipFree(p);
  if (c->own_scratch && c->scratch) (void)hipFree(c->scratch);
  c->scratch = nullptr;
  if (c->own_adj && !c->adj.empty() && c->adj[0]) (void)hipFree(c->adj[0]);
  c->adj.clear();
}

// ---------------------------------------------------------------------------
// scratch layout: every buffer of the context's scratch at a 256-byte aligned
// offset of one block; the adjoint workspace likewise
// ---------------------------------------------------------------------------
struct Sizes {
  int dim, nw, ncell, nface, nv, nvx, nvy, nblock, prec;
};

size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }

// byte sizes of the scratch buffers, in the order of scratch_slots
std::vector<size_t> scratch_sizes(const Sizes& z) {
  const size_t N = (size_t)z.ncell * z.nv, ts = z.prec == UGKS_F64 ? 8 : 4;
  return {sizeof(double) * 8 * (size_t)z.ncell,            // gW
          sizeof(double) * NREC * (size_t)z.nface,         // face records
          sizeof(double) * z.nface,                        // Gamma
          sizeof(double) * 64 * (size_t)z.ncell,           // macro record
          sizeof(double) * z.ncell,                        // macro diagonal
          sizeof(double) * z.nw * (size_t)z.ncell,         // dW*
          sizeof(double) * z.nw * (size_t)z.ncell,         // dW
          sizeof(double) * z.nw * (size_t)z.ncell,         // W'
          sizeof(double) * 4 * (size_t)z.nblock,           // residual partials
          sizeof(double) * NCREC * (size_t)z.ncell,        // cell records
          sizeof(double) * NMREC * (size_t)z.ncell,        // moment records
          ts * N, ts * N,                                  // D / r / dF* (h, b)
          sizeof(double) * z.nw * (size_t)z.nface,         // face macro flux
          sizeof(double) * flux_part_doubles(z.nv, z.nface)};  // chunk partials
}

std::vector<void**> scratch_slots(ugks_ctx* c) {
  return {&c->s_gW, &c->s_rec, &c->s_gam, &c->s_R, &c->s_Dg, &c->s_dWs, &c->s_dW, &c->s_Wp, &c->s_rpart,
          &c->s_crec, &c->s_mrec, &c->s_Dh, &c->s_Db, &c->s_F, &c->s_part};
}

size_t scratch_bytes(const Sizes& z) {
  size_t t = 0;
  for (size_t b : scratch_sizes(z)) t += align256(std::max<size_t>(b, 256));
  return t;
}

// doubles of each adjoint buffer (enum AdjBuf order, defined below)
std::vector<size_t> adjoint_counts(const Sizes& z);

size_t adjoint_bytes(const Sizes& z) {
  size_t t = 0;
  for (size_t n : adjoint_counts(z)) t += align256(sizeof(double) * std::max<size_t>(n, 1));
  return t;
}

// carve the adjoint buffers from one block
void carve_adjoint(ugks_ctx* c, const Sizes& z, char* base) {
  std::vector<size_t> n = adjoint_counts(z);
  c->adj.assign(n.size(), nullptr);
  size_t off = 0;
  for (size_t i = 0; i < n.size(); ++i) {
    c->adj[i] = base + off;
    off += align256(sizeof(double) * std::max<size_t>(n[i], 1));
  }
}

// sizes of a problem (validated by the caller)
Sizes sizes_of(const ugks_problem* p) {
  Sizes z{};
  z.dim = p->dim; z.nw = p->dim + 2; z.nv = p->nvx * ((p->dim == 2) ? p->nvy : 1);
  z.nvx = p->nvx; z.nvy = (p->dim == 2) ? p->nvy : 1;
  if (p->nvu > 0) { z.nv = p->nvu; z.nvx = p->nvu; z.nvy = 1; }
  z.nblock = p->nblock; z.prec = p->prec;
  for (int b = 0; b < p->nblock; ++b) {
    const int ni = p->bint[6 * b], nj = (p->dim == 2) ? p->bint[6 * b + 1] : 1;
    z.ncell += ni * nj;
    z.nface += (ni + 1) * nj + ((p->dim == 2) ? ni * (nj + 1) : 0);
  }
  return z;
}

Sizes sizes_of(const ugks_ctx* c) {
  return Sizes{c->dim, c->nw, c->ncell, c->nface, c->nv, c->nvx, c->nvy, (int)c->blk.size(), c->prec};
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char* ugks_last_error(void) { return g_err.c_str(); }

static int create_ctx(const ugks_problem* p, int device, void* work, size_t work_bytes, ugks_ctx** out);

int ugks_create(const ugks_problem* p, int device, ugks_ctx** out) {
  return create_ctx(p, device, nullptr, 0, out);
}

int ugks_create_with_workspace(const ugks_problem* p, int device, void* work, size_t work_bytes, ugks_ctx** out) {
  if (!work) return fail(UGKS_E_ARG, "null workspace");
  if ((uintptr_t)work % 256 != 0) return fail(UGKS_E_ARG, "workspace must be 256-byte aligned");
  return create_ctx(p, device, work, work_bytes, out);
}

static int check_problem(const ugks_problem* p) {
  if (p->dim != 1 && p->dim != 2) return fail(UGKS_E_ARG, "dim must be 1 or 2");
  if (p->prec != UGKS_F64 && p->prec != UGKS_F32) return fail(UGKS_E_ARG, "prec must be UGKS_F64 or UGKS_F32");
  if (p->nvu < 0) return fail(UGKS_E_ARG, "negative nvu");
  if (p->nvu > 0) {
    if (p->dim != 2) return fail(UGKS_E_UNSUPPORTED, "an unstructured velocity mesh is 2D");
    if (!p->vu || !p->wu) return fail(UGKS_E_ARG, "null velocity mesh");
    for (int k = 0; k < p->nvu; ++k)
      if (!(p->wu[k] > 0.0)) return fail(UGKS_E_ARG, "non-positive velocity cell area");
  } else {
    if (p->nvx < 2 || (p->dim == 2 && p->nvy < 2) || (p->dim == 1 && p->nvy != 1))
      return fail(UGKS_E_SHAPE, "bad velocity grid size");
    if (!p->vx || !p->vy) return fail(UGKS_E_ARG, "null velocity points");
  }
  if (!p->bint || !p->bdbl || !p->nodes || p->nblock < 1) return fail(UGKS_E_ARG, "null array or no block");
  for (int b = 0; b < p->nblock; ++b)
    if (p->bint[6 * b] < 2 || (p->dim == 2 && p->bint[6 * b + 1] < 2)) return fail(UGKS_E_ARG, "bad block size");
  return UGKS_OK;
}

int ugks_workspace_size(const ugks_problem* p, size_t* scratch, size_t* adjoint) {
  g_err.clear();
  if (!p) return fail(UGKS_E_ARG, "null problem");
  if (int rc = check_problem(p)) return rc;
  const Sizes z = sizes_of(p);
  if (scratch) *scratch = scratch_bytes(z);
  if (adjoint) *adjoint = adjoint_bytes(z);
  return UGKS_OK;
}

static int create_ctx(const ugks_problem* p, int device, void* work, size_t work_bytes, ugks_ctx** out) {
  g_err.clear();
  if (!p || !out) return fail(UGKS_E_ARG, "null argument");
  *out = nullptr;
  if (int rc = check_problem(p)) return rc;
  if (work) {
    const size_t need = scratch_bytes(sizes_of(p));
    if (work_bytes < need) return fail(UGKS_E_SHAPE, "workspace smaller than ugks_workspace_size's scratch bytes");
  }
  if (!(p->cfl_s > 0) || !(p->cfl_p > 0) || !(p->pr > 0)) return fail(UGKS_E_ARG, "bad CFL or Prandtl number");
  auto* c = new ugks_ctx();
  c->device = device;
  c->dim = p->dim; c->nxi = 3 - p->dim; c->nw = p->dim + 2; c->prec = p->prec;
  c->pr = p->pr; c->omega = p->omega; c->mu_ref = p->mu_ref; c->rt_ref = p->rt_ref;
  c->cfl_s = p->cfl_s; c->cfl_p = p->cfl_p;
  for (int m = 0; m < 4; ++m) c->vrange[m] = p->vrange[m];
  for (int m = 0; m < c->nw; ++m) c->winf[m] = p->winf[m];
  if (p->nvu > 0) {
    // unstructured velocity mesh: the given points and cell areas
    c->nvx = p->nvu; c->nvy = 1; c->nv = p->nvu;
    c->vx.assign(p->vu, p->vu + p->nvu);
    c->vy.assign(p->vu + p->nvu, p->vu + 2 * (size_t)p->nvu);
    c->wk.assign(p->wu, p->wu + p->nvu);
  } else {
    c->nvx = p->nvx; c->nvy = p->nvy; c->nv = p->nvx * p->nvy;
    std::vector<double> wx = nc_weights(c->nvx, p->vrange[0], p->vrange[1]);
    std::vector<double> wy = (c->dim == 2) ? nc_weights(c->nvy, p->vrange[2], p->vrange[3]) : std::vector<double>{1.0};
    c->vx.resize(c->nv); c->vy.resize(c->nv); c->wk.resize(c->nv);
    for (int iy = 0; iy < c->nvy; ++iy)
      for (int ix = 0; ix < c->nvx; ++ix) {
        int k = ix + c->nvx * iy;
        c->vx[k] = p->vx[ix];
        c->vy[k] = (c->dim == 2) ? p->vy[iy] : 0.0;
        c->wk[k] = wx[ix] * wy[iy];
      }
  }
  const double* np = p->nodes;
  int ncell = 0;
  size_t nnode = 0;
  for (int b = 0; b < p->nblock; ++b) {
    Block B;
    B.ni = p->bint[6 * b];
    B.nj = (c->dim == 2) ? p->bint[6 * b + 1] : 1;
    for (int s = 0; s < 4; ++s) B.bc[s] = p->bint[6 * b + 2 + s];
    for (int s = 0; s < 4; ++s) {
      B.rtw[s] = p->bdbl[14 * b + s];
      B.vwx[s] = p->bdbl[14 * b + 4 + s];
      B.vwy[s] = p->bdbl[14 * b + 8 + s];
    }
    B.xc0 = p->bdbl[14 * b + 12];
    B.yc0 = p->bdbl[14 * b + 13];
    bool ok = B.ni >= 2 && B.nj >= 1;
    for (int dir = 0; dir < 2; ++dir) {
      bool a = B.bc[2 * dir] == UGKS_BC_PERIODIC, e = B.bc[2 * dir + 1] == UGKS_BC_PERIODIC;
      if (a != e) ok = false;
      if (a && ((dir == 0 && B.ni < 3) || (dir == 1 && B.nj < 3))) ok = false;
    }
    for (int s = 0; s < 4; ++s) {
      if (B.bc[s] < 0 || B.bc[s] > 4) ok = false;
      if (B.bc[s] == UGKS_BC_WALL && !(B.rtw[s] > 0)) ok = false;
    }
    if (c->dim == 2 && B.nj < 2) ok = false;
    if (!ok) { delete c; return fail(UGKS_E_ARG, "bad block " + std::to_string(b)); }
    size_t nn = (size_t)(B.ni + 1) * ((c->dim == 2) ? (B.nj + 1) : 1);
    B.x0.assign(np, np + nn); np += nn;
    if (c->dim == 2) { B.y0.assign(np, np + nn); np += nn; }
    else B.y0.assign(nn, 0.0);
    B.cell0 = ncell;
    c->node0.push_back(nnode);
    ncell += B.ni * B.nj;
    nnode += nn;
    c->max_ni = std::max(c->max_ni, B.ni);
    c->max_nj = std::max(c->max_nj, B.nj);
    if (B.bc[2] == UGKS_BC_PERIODIC) c->any_pj = 1;
    if (B.bc[0] == UGKS_BC_PERIODIC) c->any_pi = 1;
    c->blk.push_back(std::move(B));
  }
  if (c->dim == 2 && c->max_nj > 512) { delete c; return fail(UGKS_E_UNSUPPORTED, "nj above 512"); }
  if (c->any_pj && c->max_ni > 256) { delete c; return fail(UGKS_E_UNSUPPORTED, "periodic j needs ni <= 256"); }
  if (micro_lds(c->dim, c->max_ni, c->max_nj, c->any_pj, 16) > 160 * 1024) {
    delete c; return fail(UGKS_E_UNSUPPORTED, "micro sweep LDS above 160 KiB");
  }
  if (macro_lds(((c->max_nj + 63) / 64) * 64, c->max_ni, c->max_nj, c->any_pi, c->any_pj) > 160 * 1024) {
    delete c; return fail(UGKS_E_UNSUPPORTED, "macro sweep LDS above 160 KiB");
  }
  c->ncell = ncell;
  c->xn.assign(nnode, 0.0);
  c->yn.assign(nnode, 0.0);
  c->cblk.resize(ncell); c->ci.resize(ncell); c->cj.resize(ncell);
  for (int b = 0; b < (int)c->blk.size(); ++b)
    for (int j = 0; j < c->blk[b].nj; ++j)
      for (int i = 0; i < c->blk[b].ni; ++i) {
        int n = cell_of(c, b, i, j);
        c->cblk[n] = b; c->ci[n] = i; c->cj[n] = j;
      }
  c->type.assign(ncell, UGKS_FIELD);
  c->vol.resize(ncell); c->ccx.resize(ncell); c->ccy.resize(ncell); c->G.resize(4 * (size_t)ncell); c->cdx.resize(8 * (size_t)ncell); c->dtp.resize(ncell);
  build_faces(c);
  build_tables(c);
  compute_geometry(c);
  // device
  if (hipSetDevice(device) != hipSuccess) { delete c; return fail(UGKS_E_DEVICE, "hipSetDevice failed"); }
  {
    static std::vector<int> ready;  // devices whose kernel attributes are set
    if (std::find(ready.begin(), ready.end(), device) == ready.end()) {
      if (init_kernel_attributes()) { delete c; return fail(UGKS_E_DEVICE, "kernel attributes"); }
      ready.push_back(device);
    }
  }
  // the static scratch of ugks_flux_noalloc: its address on this device
  if (static_scratch(device, &c->sscratch)) c->sscratch = nullptr;
  int rc = UGKS_OK;
  std::vector<int> binfo(8 * c->blk.size(), 0);
  for (size_t b = 0; b < c->blk.size(); ++b) {
    const Block& B = c->blk[b];
    binfo[8 * b] = B.ni; binfo[8 * b + 1] = B.nj; binfo[8 * b + 2] = B.cell0;
    binfo[8 * b + 3] = B.bc[0] == UGKS_BC_PERIODIC; binfo[8 * b + 4] = B.bc[2] == UGKS_BC_PERIODIC;
  }
  if (!rc) rc = upload(c->d_vx, c->vx);
  if (!rc) rc = upload(c->d_vy, c->vy);
  if (!rc) rc = upload(c->d_wk, c->wk);
  if (!rc) rc = upload(c->d_cf, c->cf);
  if (!rc) rc = upload(c->d_fcell, c->fcell);
  if (!rc) rc = upload(c->d_binfo, binfo);
  if (!rc) rc = upload_farfield(c);
  if (!rc) rc = upload_geometry(c);
  if (!rc) rc = upload_tables(c);
  // face range of each block (faces are numbered block by block)
  c->bface.assign(c->blk.size() + 1, 0);
  for (size_t b = 0; b < c->blk.size(); ++b)
    c->bface[b + 1] = (b + 1 < c->blk.size()) ? c->blk[b + 1].face_i0 : c->nface;
  if (!rc) rc = upload(c->d_bface, c->bface);
  if (!rc) rc = alloc(c->d_side, sizeof(double) * 16 * c->blk.size());
  if (!rc) {
    void* st = nullptr;
    rc = alloc(st, sizeof(unsigned));
    c->d_status = (unsigned*)st;
  }
  if (!rc && hipMemset(c->d_status, 0, sizeof(unsigned)) != hipSuccess) rc = fail(UGKS_E_DEVICE, "hipMemset failed");
  // scratch: the caller's workspace or one allocation; with a workspace
  // large enough, the adjoint workspace follows the scratch in it
  const Sizes z = sizes_of(c);
  const size_t sbytes = scratch_bytes(z);
  if (!rc) {
    if (work) {
      c->scratch = work;
      c->own_scratch = false;
      if (work_bytes >= sbytes + adjoint_bytes(z)) {
        carve_adjoint(c, z, (char*)work + sbytes);
        c->own_adj = false;
      }
    } else if (hipMalloc(&c->scratch, sbytes) != hipSuccess) {
      c->scratch = nullptr;
      rc = fail(UGKS_E_DEVICE, "scratch allocation");
    }
  }
  if (!rc) {
    std::vector<size_t> sz = scratch_sizes(z);
    std::vector<void**> slot = scratch_slots(c);
    size_t off = 0;
    for (size_t i = 0; i < sz.size(); ++i) {
      *slot[i] = (char*)c->scratch + off;
      off += align256(std::max<size_t>(sz[i], 256));
    }
  }
  if (rc) { free_all(c); delete c; return rc; }
  // scratch that kernels read before writing everywhere starts at zero
  if (hipMemset(c->s_rec, 0, sizeof(double) * NREC * (size_t)c->nface) != hipSuccess ||
      hipMemset(c->s_mrec, 0, sizeof(double) * NMREC * (size_t)c->ncell) != hipSuccess ||
      hipMemset(c->s_crec, 0, sizeof(double) * NCREC * (size_t)c->ncell) != hipSuccess) {
    free_all(c); delete c; return fail(UGKS_E_DEVICE, "hipMemset failed");
  }
  fill_dev(c);
  c->dev.status = c->d_status;
  // default launch shapes (measured on the cylinder workload; ugks_autotune
  // refines them per case): the FP64 flux pass keeps more registers per
  // wavefront with six core rows per workgroup
  c->dev.kc_max = 16;
  c->dev.rg_eq = 8;
  c->dev.rg_flux = 8;
  *out = c;
  return UGKS_OK;
}

int ugks_destroy(ugks_ctx* c) {
  if (!c) return UGKS_OK;
  (void)hipDeviceSynchronize();
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->cap) (void)hipStreamDestroy(c->cap);
  free_all(c);
  delete c;
  return UGKS_OK;
}

int ugks_sizes(const ugks_ctx* c, int32_t* ncell, int32_t* nface, int32_t* nv, int32_t* prec) {
  if (!c) return fail(UGKS_E_ARG, "null context");
  if (ncell) *ncell = c->ncell;
  if (nface) *nface = c->nface;
  if (nv) *nv = c->nv;
  if (prec) *prec = c->prec;
  return UGKS_OK;
}

int ugks_set_poses(ugks_ctx* c, const double* poses, double* dts) {
  if (!c || !poses) return fail(UGKS_E_ARG, "null argument");
  ++c->version;
  for (size_t b = 0; b < c->blk.size(); ++b)
    for (int m = 0; m < 6; ++m) {
      if (!std::isfinite(poses[6 * b + m])) return fail(UGKS_E_ARG, "non-finite pose");
    }
  for (size_t b = 0; b < c->blk.size(); ++b)
    for (int m = 0; m < 6; ++m) c->blk[b].pose[m] = poses[6 * b + m];
  compute_geometry(c);
  int rc = upload_geometry(c);
  if (rc) return rc;
  if (dts) *dts = c->dts;
  return UGKS_OK;
}

// face data recomputed after a change of block velocities or wall
// temperatures, keeping the time steps dt_s and dt' of the last pose
static int refresh_frozen_steps(ugks_ctx* c) {
  const double dts = c->dts;
  const std::vector<double> dtp = c->dtp;
  compute_geometry(c);
  c->dts = dts;
  c->dtp = dtp;
  return upload_geometry(c);
}

int ugks_set_wall_rt(ugks_ctx* c, int32_t blk, int32_t side, double rtw) {
  if (!c) return fail(UGKS_E_ARG, "null context");
  if (blk < 0 || blk >= (int)c->blk.size() || side < 0 || side > 3) return fail(UGKS_E_ARG, "bad block side");
  if (!(rtw > 0.0) || !std::isfinite(rtw)) return fail(UGKS_E_ARG, "wall RT must be positive");
  ++c->version;
  c->blk[blk].rtw[side] = rtw;
  return refresh_frozen_steps(c);
}

int ugks_set_farfield(ugks_ctx* c, const double* winf) {
  if (!c || !winf) return fail(UGKS_E_ARG, "null argument");
  double w[4] = {0, 0, 0, 0};
  for (int m = 0; m < c->nw; ++m) {
    if (!std::isfinite(winf[m])) return fail(UGKS_E_ARG, "non-finite far-field state");
    w[m] = winf[m];
  }
  double ke = 0.0;
  for (int d = 0; d < c->dim; ++d) ke += 0.5 * w[1 + d] * w[1 + d] / w[0];
  if (!(w[0] > 0.0) || !(w[c->dim + 1] - ke > 0.0)) return fail(UGKS_E_ARG, "far-field density and internal energy must be positive");
  HIPCHK(hipDeviceSynchronize());  // kernels in flight read the old Maxwellian
  for (int m = 0; m < 4; ++m) c->winf[m] = w[m];
  ++c->version;  // captured graphs hold the far-field state
  int rc = upload_farfield(c);
  if (!rc) fill_dev(c);
  return rc;
}

int ugks_set_block_velocity(ugks_ctx* c, int32_t blk, double ux, double uy, double om) {
  if (!c) return fail(UGKS_E_ARG, "null context");
  if (blk < 0 || blk >= (int)c->blk.size()) return fail(UGKS_E_ARG, "bad block");
  if (!std::isfinite(ux) || !std::isfinite(uy) || !std::isfinite(om)) return fail(UGKS_E_ARG, "non-finite velocity");
  ++c->version;
  c->blk[blk].pose[3] = ux;
  c->blk[blk].pose[4] = uy;
  c->blk[blk].pose[5] = om;
  return refresh_frozen_steps(c);
}

int ugks_face_geometry(const ugks_ctx* c, double* fgeo) {
  if (!c || !fgeo) return fail(UGKS_E_ARG, "null argument");
  std::memcpy(fgeo, c->fgeo.data(), sizeof(double) * 8 * (size_t)c->nface);
  return UGKS_OK;
}

int ugks_overset_rows(const ugks_ctx* c, int32_t* nrec, int32_t* nrefill, int32_t* pending) {
  if (!c) return fail(UGKS_E_ARG, "null context");
  if (nrec) *nrec = c->nrec;
  if (nrefill) *nrefill = (int32_t)c->h_rec.size() - c->nrec;
  if (pending) *pending = (c->nref > 0) ? 1 : 0;
  return UGKS_OK;
}

int ugks_last_flux(const ugks_ctx* c, double* F, void* stream) {
  if (!c || !F) return fail(UGKS_E_ARG, "null argument");
  HIPCHK(hipMemcpyAsync(F, c->s_F, sizeof(double) * c->nw * (size_t)c->nface, hipMemcpyDeviceToDevice,
                        (hipStream_t)stream));
  return UGKS_OK;
}

int ugks_timesteps(const ugks_ctx* c, double* dts, double* dtp) {
  if (!c) return fail(UGKS_E_ARG, "null context");
  if (dts) *dts = c->dts;
  if (dtp) std::memcpy(dtp, c->dtp.data(), sizeof(double) * c->ncell);
  return UGKS_OK;
}

int ugks_set_types(ugks_ctx* c, const int8_t* types) {
  if (!c || !types) return fail(UGKS_E_ARG, "null argument");
  ++c->version;
  for (int n = 0; n < c->ncell; ++n)
    if (types[n] < 0 || types[n] > 2) return fail(UGKS_E_ARG, "bad cell kind");
  c->type.assign(types, types + c->ncell);
  build_tables(c);
  compute_geometry(c);  // dt_s is a minimum over field cells
  int rc = upload_tables(c);
  if (!rc) rc = upload_geometry(c);
  if (!rc) fill_dev(c);
  return rc;
}

int ugks_get_types(const ugks_ctx* c, int8_t* types) {
  if (!c || !types) return fail(UGKS_E_ARG, "null argument");
  std::memcpy(types, c->type.data(), c->ncell);
  return UGKS_OK;
}

// donor table of nrow rows (the first nrec are receptors) to host and device
static int install_overset(ugks_ctx* c, int nrow, int nrec, const int32_t* rec, const int32_t* ptr,
                           const int32_t* don, const double* w) {
  ++c->version;
  c->nrec = nrec;
  c->nref = nrow - nrec;
  c->h_rec.assign(rec, rec + nrow);
  c->h_ptr.assign(ptr, ptr + nrow + 1);
  const int nd = nrow > 0 ? ptr[nrow] : 0;
  c->h_don.assign(don, don + nd);
  c->h_w.assign(w, w + nd);
  for (void** p : {&c->d_rec, &c->d_ptr, &c->d_don, &c->d_w})
    if (*p) { (void)hipFree(*p); *p = nullptr; }
  int rc = upload(c->d_rec, c->h_rec);
  if (!rc) rc = upload(c->d_ptr, c->h_ptr);
  if (!rc) rc = upload(c->d_don, c->h_don);
  if (!rc) rc = upload(c->d_w, c->h_w);
  return rc;
}

int ugks_set_overset(ugks_ctx* c, int32_t nrec, const int32_t* rec, const int32_t* ptr, const int32_t* don,
                     const double* w) {
  if (!c || nrec < 0) return fail(UGKS_E_ARG, "bad argument");
  if (nrec > 0 && (!rec || !ptr || !don || !w)) return fail(UGKS_E_ARG, "null overset array");
  if (nrec > 0) {
    if (ptr[0] != 0) return fail(UGKS_E_ARG, "ptr[0] must be 0");
    for (int r = 0; r < nrec; ++r) {
      if (rec[r] < 0 || rec[r] >= c->ncell) return fail(UGKS_E_ARG, "receptor out of range");
      if (ptr[r + 1] < ptr[r]) return fail(UGKS_E_ARG, "ptr not monotone");
    }
    for (int p = 0; p < ptr[nrec]; ++p) {
      if (don[p] < 0 || don[p] >= c->ncell) return fail(UGKS_E_ARG, "donor out of range");
      if (c->type[don[p]] != UGKS_FIELD) return fail(UGKS_E_ARG, "donor is not a field cell");
    }
  }
  return install_overset(c, nrec, nrec, rec, ptr, don, w);
}

int ugks_get_overset(const ugks_ctx* c, int32_t* nrec, int32_t* ndon, int32_t* rec, int32_t* ptr, int32_t* don,
                     double* w) {
  if (!c) return fail(UGKS_E_ARG, "null context");
  const int nd = c->nrec > 0 ? c->h_ptr[c->nrec] : 0;
  if (nrec) *nrec = c->nrec;
  if (ndon) *ndon = nd;
  if (rec && c->nrec) std::memcpy(rec, c->h_rec.data(), sizeof(int32_t) * c->nrec);
  if (ptr) {
    if (c->nrec) std::memcpy(ptr, c->h_ptr.data(), sizeof(int32_t) * (c->nrec + 1));
    else ptr[0] = 0;
  }
  if (don && nd) std::memcpy(don, c->h_don.data(), sizeof(int32_t) * nd);
  if (w && nd) std::memcpy(w, c->h_w.data(), sizeof(double) * nd);
  return UGKS_OK;
}

static int assemble_impl(ugks_ctx* c, int32_t wrule, int32_t overlap, int32_t* nrec, bool device);

int overset_assemble(ugks_ctx* c, int32_t wrule, int32_t overlap, int32_t* nrec) {
  return assemble_impl(c, wrule, overlap, nrec, false);
}

int overset_assemble_device(ugks_ctx* c, int32_t wrule, int32_t overlap, int32_t* nrec) {
  return assemble_impl(c, wrule, overlap, nrec, true);
}

static int assemble_impl(ugks_ctx* c, int32_t wrule, int32_t overlap, int32_t* nrec, bool device) {
  if (!c) return fail(UGKS_E_ARG, "null context");
  ++c->version;
  if (wrule != 0 && wrule != 1) return fail(UGKS_E_ARG, "wrule must be 0 or 1");
  if (overlap < 0) return fail(UGKS_E_ARG, "negative overlap");
  if (c->dim != 2) return fail(UGKS_E_UNSUPPORTED, "overset assembly is 2D");
  OversetInput in;
  in.nblock = (int)c->blk.size();
  for (const auto& B : c->blk) {
    in.ni.push_back(B.ni); in.nj.push_back(B.nj); in.cell0.push_back(B.cell0);
    for (int s = 0; s < 4; ++s) in.bc.push_back(B.bc[s]);
  }
  in.xn = &c->xn; in.yn = &c->yn; in.node0 = &c->node0;
  in.cx = &c->ccx; in.cy = &c->ccy; in.vol = &c->vol;
  in.old_type = &c->type;
  OversetOutput res;
  std::string msg;
  int rc = UGKS_OK;
  if (device) {
    if (hipSetDevice(c->device) != hipSuccess) return fail(UGKS_E_DEVICE, "hipSetDevice failed");
    rc = overset_build_device(in, wrule, overlap, res, msg);
  } else {
    rc = overset_build(in, wrule, overlap, res, msg);
  }
  if (rc) return fail(rc, msg);
  c->type = res.type;
  build_tables(c);
  compute_geometry(c);
  rc = upload_tables(c);
  if (!rc) rc = upload_geometry(c);
  if (!rc) fill_dev(c);
  if (rc) return rc;
  rc = install_overset(c, (int)res.rec.size(), res.nrec, res.rec.data(), res.ptr.data(), res.don.data(),
                       res.w.data());
  if (!rc && nrec) *nrec = res.nrec;
  return rc;
}

static int check_dev(const ugks_ctx* c, std::initializer_list<const void*> ps) {
  if (!c) return fail(UGKS_E_ARG, "null context");
  for (const void* p : ps)
    if (!p) return fail(UGKS_E_ARG, "null device array");
  return UGKS_OK;
}

int ugks_maxwellian(ugks_ctx* c, const double* W, void* h, void* b, void* stream) {
  if (int rc = check_dev(c, {W, h, b})) return rc;
  launch_maxwellian(c->dev, c->prec, W, h, b, (hipStream_t)stream);
  HIPCHK(hipGetLastError());
  return UGKS_OK;
}

int ugks_moments(ugks_ctx* c, const void* h, const void* b, double* W, double* q, void* stream) {
  if (int rc = check_dev(c, {h, b, W, q})) return rc;
  launch_moments(c->dev, c->prec, h, b, W, q, (hipStream_t)stream);
  HIPCHK(hipGetLastError());
  return UGKS_OK;
}

int ugks_heatflux(ugks_ctx* c, const void* h, const void* b, const double* W, double* q, void* stream) {
  if (int rc = check_dev(c, {h, b, W, q})) return rc;
  launch_step7(c->dev, c->prec, 2, h, b, nullptr, nullptr, const_cast<double*>(W), q, (double*)c->s_mrec,
               (hipStream_t)stream);
  HIPCHK(hipGetLastError());
  return UGKS_OK;
}

int ugks_flux(ugks_ctx* c, double dts, const void* h, const void* b, const double* W, const double* q,
              void* Dh, void* Db, double* F, double* wall, void* stream) {
  if (int rc = check_dev(c, {h, b, W, q, Dh, Db})) return rc;
  if (!(dts > 0) || !std::isfinite(dts)) return fail(UGKS_E_ARG, "dts must be positive");
  hipStream_t st = (hipStream_t)stream;
  if (wall) launch_fill(wall, (c->nw + 1) * (size_t)c->nface, 0.0, st);
  double* Fo = F ? F : (double*)c->s_F;
  launch_fill(Fo, c->nw * (size_t)c->nface, 0.0, st);
  launch_flux(c->dev, c->prec, (const int*)c->d_binfo, c->max_nj, dts, h, b, W, q, (double*)c->s_gW,
              (double*)c->s_rec, (double*)c->s_part, Dh, Db, Fo, wall, st);
  HIPCHK(hipGetLastError());
  return UGKS_OK;
}

int ugks_flux_noalloc(ugks_ctx* c, double dts, const void* h, const void* b, const double* W, const double* q,
                      void* Dh, void* Db, double* F, double* wall, void* stream) {
  if (int rc = check_dev(c, {h, b, W, q, Dh, Db})) return rc;
  if (!(dts > 0) || !std::isfinite(dts)) return fail(UGKS_E_ARG, "dts must be positive");
  if (!c->sscratch) return fail(UGKS_E_DEVICE, "the static scratch array has no address on this device");
  // the flux's scratch carved from the static array: W gradients, face
  // records, chunk partial sums, and the face macro flux when F is NULL
  const size_t sz[4] = {sizeof(double) * 8 * (size_t)c->ncell, sizeof(double) * NREC * (size_t)c->nface,
                        sizeof(double) * flux_part_doubles(c->nv, c->nface),
                        F ? 0 : sizeof(double) * c->nw * (size_t)c->nface};
  size_t off[4], total = 0;
  for (int i = 0; i < 4; ++i) { off[i] = total; total += (sz[i] + 255) & ~(size_t)255; }
  if (total > kStaticScratchBytes)
    return fail(UGKS_E_SHAPE, "ugks_flux_noalloc needs " + std::to_string(total) + " bytes of scratch, above its " +
                                  std::to_string(kStaticScratchBytes) + "-byte static array");
  char* base = (char*)c->sscratch;
  double* gW = (double*)(base + off[0]);
  double* rec = (double*)(base + off[1]);
  double* part = (double*)(base + off[2]);
  double* Fo = F ? F : (double*)(base + off[3]);
  hipStream_t st = (hipStream_t)stream;
  // the array keeps the last call's contents: the face records start at zero
  // like the context's (fill kernels, no memset)
  launch_fill(rec, NREC * (size_t)c->nface, 0.0, st);
  if (wall) launch_fill(wall, (c->nw + 1) * (size_t)c->nface, 0.0, st);
  launch_fill(Fo, c->nw * (size_t)c->nface, 0.0, st);
  launch_flux(c->dev, c->prec, (const int*)c->d_binfo, c->max_nj, dts, h, b, W, q, gW, rec, part, Dh, Db, Fo, wall,
              st);
  HIPCHK(hipGetLastError());
  return UGKS_OK;
}

int overset_interp(ugks_ctx* c, void* h, void* b, double* W, double* q, void* stream) {
  if (int rc = check_dev(c, {h, b, W, q})) return rc;
  launch_interp(c->dev, c->prec, c->nrec, (const int*)c->d_rec, (const int*)c->d_ptr, (const int*)c->d_don,
                (const double*)c->d_w, h, b, W, q, (hipStream_t)stream);
  HIPCHK(hipGetLastError());
  return UGKS_OK;
}

int ugks_begin_step(ugks_ctx* c, double dt, void* h, void* b, double* W, double* q, void* Sh, void* Sb,
                    double* Fn, void* stream) {
  if (int rc = check_dev(c, {h, b, W, q, Sh, Sb, Fn})) return rc;
  if (!(dt > 0) || !std::isfinite(dt)) return fail(UGKS_E_ARG, "dt must be positive");
  hipStream_t st = (hipStream_t)stream;
  // once after an assembly the cells uncovered from holes (rows after the
  // receptors; their donors were live cells), then the receptors, which may
  // use them as donors
  if (c->nref > 0)
    launch_interp(c->dev, c->prec, c->nref, (const int*)c->d_rec + c->nrec, (const int*)c->d_ptr + c->nrec,
                  (const int*)c->d_don, (const double*)c->d_w, h, b, W, q, st);
  c->nref = 0;
  launch_interp(c->dev, c->prec, c->nrec, (const int*)c->d_rec, (const int*)c->d_ptr, (const int*)c->d_don,
                (const double*)c->d_w, h, b, W, q, st);
  launch_fill(Fn, c->nw * (size_t)c->nface, 0.0, st);
  // the level-n divergence is staged in Sh, Sb
  launch_flux(c->dev, c->prec, (const int*)c->d_binfo, c->max_nj, c->dts, h, b, W, q, (double*)c->s_gW,
              (double*)c->s_rec, (double*)c->s_part, Sh, Sb, Fn, nullptr, st);
  launch_cellrec(c->dev, dt, W, q, nullptr, (double*)c->s_crec, st);
  launch_source(c->dev, c->prec, dt, h, b, (const double*)c->s_crec, Sh, Sb, st);
  HIPCHK(hipGetLastError());
  return c->sync_check ? ugks_status(c, stream) : UGKS_OK;
}

// the pseudo-iteration loop; with ev (9 events per inner iteration) the
// stage boundaries are recorded on the stream
static int run_inner(ugks_ctx* c, double dt, int32_t n_inner, void* h, void* b, double* W, const double* Wn,
                     double* q, const void* Sh, const void* Sb, const double* Fn, double* resid, hipStream_t st,
                     std::vector<hipEvent_t>* ev) {
  const Dev& g = c->dev;
  double* F = (double*)c->s_F;
  // moments of f^s about the velocity of W^s (heat flux source of the first
  // micro step)
  launch_step7(g, c->prec, 0, h, b, nullptr, nullptr, W, q, (double*)c->s_mrec, st);
  for (int s = 0; s < n_inner; ++s) {
    hipEvent_t* e = ev ? &(*ev)[(UGKS_NSTAGE + 1) * (size_t)s] : nullptr;
    if (e) HIPCHK(hipEventRecord(e[0], st));
    launch_interp(g, c->prec, c->nrec, (const int*)c->d_rec, (const int*)c->d_ptr, (const int*)c->d_don,
                  (const double*)c->d_w, h, b, W, q, st);
    if (e) HIPCHK(hipEventRecord(e[1], st));
    launch_flux(g, c->prec, (const int*)c->d_binfo, c->max_nj, c->dts, h, b, W, q, (double*)c->s_gW,
                (double*)c->s_rec, (double*)c->s_part, c->s_Dh, c->s_Db, F, nullptr, st, e ? e + 2 : nullptr);
    if (e) HIPCHK(hipEventRecord(e[6], st));
    launch_macro(g, (const int*)c->d_binfo, c->max_ni, c->max_nj, c->any_pi, c->any_pj, dt, W, Wn, F, Fn,
                 (double*)c->s_gam, (double*)c->s_R,
                 (double*)c->s_Dg, (double*)c->s_dWs, (double*)c->s_dW, (double*)c->s_Wp, (double*)c->s_rpart,
                 resid ? resid + (size_t)s * c->nw : nullptr, st);
    if (e) HIPCHK(hipEventRecord(e[7], st));
    launch_cellrec(g, dt, (const double*)c->s_Wp, nullptr, (const double*)c->s_mrec, (double*)c->s_crec, st);
    if (e) HIPCHK(hipEventRecord(e[8], st));
    launch_micro(g, c->prec, (const int*)c->d_binfo, c->max_ni, c->max_nj, c->any_pj, dt,
                 (const double*)c->s_crec, h, b, Sh, Sb, c->s_Dh, c->s_Db, st, e ? e + 9 : nullptr);
    if (e) HIPCHK(hipEventRecord(e[10], st));
    launch_step7(g, c->prec, 1, h, b, (const double*)c->s_crec, (const double*)c->s_Wp, W, q,
                 (double*)c->s_mrec, st);
    if (e) HIPCHK(hipEventRecord(e[11], st));
  }
  HIPCHK(hipGetLastError());
  return UGKS_OK;
}

int ugks_step(ugks_ctx* c, double dt, int32_t n_inner, void* h, void* b, double* W, const double* Wn, double* q,
              const void* Sh, const void* Sb, const double* Fn, double* resid, void* stream) {
  if (int rc = check_dev(c, {h, b, W, Wn, q, Sh, Sb, Fn})) return rc;
  if (!(dt > 0) || !std::isfinite(dt)) return fail(UGKS_E_ARG, "dt must be positive");
  if (n_inner < 0) return fail(UGKS_E_ARG, "n_inner must be >= 0");
  int rc = run_inner(c, dt, n_inner, h, b, W, Wn, q, Sh, Sb, Fn, resid, (hipStream_t)stream, nullptr);
  if (!rc && c->sync_check) rc = ugks_status(c, stream);
  return rc;
}

int ugks_step_profile(ugks_ctx* c, double dt, int32_t n_inner, void* h, void* b, double* W, const double* Wn,
                      double* q, const void* Sh, const void* Sb, const double* Fn, double* stage_ms,
                      void* stream) {
  if (int rc = check_dev(c, {h, b, W, Wn, q, Sh, Sb, Fn, stage_ms})) return rc;
  if (!(dt > 0) || !std::isfinite(dt)) return fail(UGKS_E_ARG, "dt must be positive");
  if (n_inner < 1) return fail(UGKS_E_ARG, "n_inner must be >= 1");
  hipStream_t st = (hipStream_t)stream;
  std::vector<hipEvent_t> ev((UGKS_NSTAGE + 1) * (size_t)n_inner);
  for (auto& e : ev) HIPCHK(hipEventCreate(&e));
  int rc = run_inner(c, dt, n_inner, h, b, W, Wn, q, Sh, Sb, Fn, nullptr, st, &ev);
  if (!rc) {
    if (hipEventSynchronize(ev.back()) != hipSuccess) rc = fail(UGKS_E_DEVICE, "event synchronisation failed");
  }
  if (!rc) {
    for (int k = 0; k < UGKS_NSTAGE; ++k) stage_ms[k] = 0.0;
    for (int s = 0; s < n_inner; ++s)
      for (int k = 0; k < UGKS_NSTAGE; ++k) {
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, ev[(UGKS_NSTAGE + 1) * (size_t)s + k], ev[(UGKS_NSTAGE + 1) * (size_t)s + k + 1]);
        stage_ms[k] += ms / n_inner;
      }
  }
  for (auto& e : ev) (void)hipEventDestroy(e);
  return rc;
}

// ---------------------------------------------------------------------------
// captured pseudo-iterations, batches of cases, launch-shape tuning
// ---------------------------------------------------------------------------
}  // extern "C"

namespace {

std::vector<uint64_t> step_key(const ugks_ctx* c, double dt, int n_inner, std::initializer_list<const void*> ps) {
  uint64_t bits;
  std::memcpy(&bits, &dt, sizeof bits);
  std::vector<uint64_t> k = {bits, (uint64_t)n_inner, c->version, (uint64_t)(uintptr_t)c,
                             (uint64_t)(c->dev.kc_max | (c->dev.rg_eq << 8) | (c->dev.rg_flux << 16))};
  for (const void* p : ps) k.push_back((uint64_t)(uintptr_t)p);
  return k;
}

// instantiate `graph` into *exec, updating an existing executable in place
// when the topology allows it
int graph_to_exec(hipGraph_t graph, hipGraphExec_t* exec) {
  if (*exec) {
    hipGraphNode_t err_node = nullptr;
    hipGraphExecUpdateResult res;
    if (hipGraphExecUpdate(*exec, graph, &err_node, &res) == hipSuccess && res == hipGraphExecUpdateSuccess)
      return UGKS_OK;
    (void)hipGetLastError();
    (void)hipGraphExecDestroy(*exec);
    *exec = nullptr;
  }
  if (hipGraphInstantiate(exec, graph, nullptr, nullptr, 0) != hipSuccess) {
    *exec = nullptr;
    return fail(UGKS_E_DEVICE, "hipGraphInstantiate failed");
  }
  return UGKS_OK;
}

struct StepArgs {
  double dt;
  void *h, *b;
  double* W;
  const double* Wn;
  double* q;
  const void *Sh, *Sb;
  const double* Fn;
  double* resid;
};

}  // namespace

struct ugks_batch {
  std::vector<ugks_ctx*> ctx;
  std::vector<hipStream_t> st;  // private capture streams (branches of the graph)
  std::vector<hipEvent_t> ev;   // fork and join events
  hipGraphExec_t gexec = nullptr;
  std::vector<uint64_t> gkey;
  // 1: one launch per stage for all cases (BatchPlan); 0: each case's own
  // kernel chain, the chains on concurrent branches
  int mode = 1;
  // mode 1: the cases in groups of like block height (one group per
  // branch), each group one chain of batched launches with its own plan
  std::vector<BatchPlan> plan;
  std::vector<void*> d_plan;  // device tables of each group's plan
  std::vector<size_t> plan_bytes;
};

namespace {

// one launch per stage applies to 2D cases of one storage type
bool batch_fusable(const ugks_batch* B) {
  for (const ugks_ctx* c : B->ctx)
    if (c->dim != 2 || c->prec != B->ctx[0]->prec) return false;
  return true;
}

// builds the launch plan of a batch (case table, workgroup prefix tables,
// work items sorted by decreasing cost) and uploads it; the caller has
// waited for the device
int batch_build_plan(ugks_batch* B, int grp, const std::vector<int>& members, const double* dt, void* const* h,
                     void* const* b, double* const* W, const double* const* Wn, double* const* q,
                     const void* const* Sh, const void* const* Sb, const double* const* Fn, double* const* resid) {
  const int n = (int)members.size();
  BatchPlan& P = B->plan[grp];
  P = BatchPlan{};
  P.ncase = n;
  P.prec = B->ctx[0]->prec;
  std::vector<BatchCase> cs(n);
  std::vector<int> off[5];
  for (auto& o : off) o.assign(n + 1, 0);
  // the widest micro-sweep chunk that the batch's tallest block allows (the
  // cases' own tuned chunk widths are for their own launches)
  const int kc_max = 16;
  for (int i = 0; i < n; ++i) {
    const ugks_ctx* c = B->ctx[members[i]];
    P.max_ni = std::max(P.max_ni, c->max_ni);
    P.max_nj = std::max(P.max_nj, c->max_nj);
    P.any_pi |= c->any_pi;
    P.any_pj |= c->any_pj;
  }
  micro_shape(2, P.max_ni, P.max_nj, P.any_pj, kc_max, P.micro_kc, P.micro_rows);
  if (P.micro_kc <= 0) return fail(UGKS_E_UNSUPPORTED, "no micro sweep shape fits the batch's largest block");
  P.micro_nslot = P.max_nj;
  P.micro_lds = micro_lds(2, P.max_ni, P.max_nj, P.any_pj, kc_max);
  P.macro_nt = ((P.max_nj + 63) / 64) * 64;
  P.macro_lds = macro_lds(P.macro_nt, P.max_ni, P.max_nj, P.any_pi, P.any_pj);
  // march rows per workgroup: the value most of the group's pairs were
  // tuned for (ugks_autotune on each case), per pass
  for (int m = 0; m < 2; ++m) {
    double votes[3] = {0, 0, 0};  // 6, 8, 10
    for (int i = 0; i < n; ++i) {
      const ugks_ctx* c = B->ctx[members[i]];
      const int r = m ? c->dev.rg_flux : c->dev.rg_eq;
      votes[(r == 6) ? 0 : (r == 10) ? 2 : 1] += (double)c->ncell * c->nv;
    }
    P.rg[m] = (votes[0] > votes[1] && votes[0] >= votes[2]) ? 6 : (votes[2] > votes[1]) ? 10 : 8;
  }
  std::vector<std::pair<long long, BatchItem>> mi[2], ui;
  for (int i = 0; i < n; ++i) {
    const int u = members[i];
    ugks_ctx* c = B->ctx[u];
    BatchCase& a = cs[i];
    a.g = c->dev;
    a.binfo = (const int*)c->d_binfo;
    a.nchunk = (c->nv + 63) / 64;
    a.nrec = c->nrec;
    a.dt = dt[u];
    a.dts = c->dts;
    a.h = h[u]; a.b = b[u]; a.Dh = c->s_Dh; a.Db = c->s_Db; a.Sh = Sh[u]; a.Sb = Sb[u];
    a.W = W[u]; a.q = q[u]; a.resid = resid ? resid[u] : nullptr; a.Wn = Wn[u]; a.Fn = Fn[u];
    a.gW = (double*)c->s_gW; a.rec = (double*)c->s_rec; a.part = (double*)c->s_part; a.F = (double*)c->s_F;
    a.gam = (double*)c->s_gam; a.mac = (double*)c->s_R; a.dWs = (double*)c->s_dWs; a.dW = (double*)c->s_dW;
    a.Wp = (double*)c->s_Wp; a.rpart = (double*)c->s_rpart; a.crec = (double*)c->s_crec;
    a.mrec = (double*)c->s_mrec;
    a.orec = (const int*)c->d_rec; a.optr = (const int*)c->d_ptr; a.odon = (const int*)c->d_don;
    a.ow = (const double*)c->d_w;
    if (a.resid) P.want_resid = 1;
    const int cnt[5] = {(c->ncell + 63) / 64, (c->nface + 63) / 64, (c->ncell + 3) / 4, (c->nrec + 3) / 4,
                        (int)c->blk.size()};
    for (int k = 0; k < 5; ++k) off[k][i + 1] = off[k][i] + cnt[k];
    const int nchu = (c->nv + P.micro_kc - 1) / P.micro_kc;
    for (int z = 0; z < (int)c->blk.size(); ++z) {
      const Block& bl = c->blk[z];
      for (int m = 0; m < 2; ++m)
        for (int y = 0; y * P.rg[m] < bl.nj; ++y) {
          const long long cost = (long long)bl.ni * std::min(P.rg[m], bl.nj - y * P.rg[m]);
          for (int x = 0; x < a.nchunk; ++x) mi[m].push_back({cost, BatchItem{i, x, y, z}});
        }
      const long long ucost = (long long)(bl.ni + bl.nj) * 1024 + bl.nj;
      for (int x = 0; x < nchu; ++x) ui.push_back({ucost, BatchItem{i, x, z, 0}});
    }
  }
  auto by_cost = [](const std::pair<long long, BatchItem>& l, const std::pair<long long, BatchItem>& r) {
    return l.first > r.first;
  };
  for (auto& v : mi) std::stable_sort(v.begin(), v.end(), by_cost);
  std::stable_sort(ui.begin(), ui.end(), by_cost);
  P.n_cell64 = off[0][n]; P.n_face64 = off[1][n]; P.n_cell4 = off[2][n]; P.n_rec4 = off[3][n];
  P.n_block = off[4][n];
  P.n_micro = (int)ui.size();
  for (int m = 0; m < 2; ++m) {
    P.n_march[m] = (int)mi[m].size();
    if (batch_march_grid(P.prec, P.rg[m], m, P.grid_march[m])) return fail(UGKS_E_DEVICE, "occupancy query failed");
    P.grid_march[m] = std::min(P.grid_march[m], std::max(P.n_march[m], 1));
  }
  if (batch_micro_grid(P.micro_lds, P.grid_micro)) return fail(UGKS_E_DEVICE, "occupancy query failed");
  P.grid_micro = std::min(P.grid_micro, std::max(P.n_micro, 1));
  // one device block: cases, five prefix tables, the items of both march
  // passes and of the micro sweep
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t s_cs = al(sizeof(BatchCase) * n), s_off = al(sizeof(int) * (n + 1));
  const size_t s_it[3] = {al(sizeof(BatchItem) * std::max<size_t>(mi[0].size(), 1)),
                          al(sizeof(BatchItem) * std::max<size_t>(mi[1].size(), 1)),
                          al(sizeof(BatchItem) * std::max<size_t>(ui.size(), 1))};
  const size_t total = s_cs + 5 * s_off + s_it[0] + s_it[1] + s_it[2];
  if (total > B->plan_bytes[grp]) {
    if (B->d_plan[grp]) (void)hipFree(B->d_plan[grp]);
    B->d_plan[grp] = nullptr;
    B->plan_bytes[grp] = 0;
    if (hipMalloc(&B->d_plan[grp], total) != hipSuccess)
      return fail(UGKS_E_DEVICE, "hipMalloc of the batch plan failed");
    B->plan_bytes[grp] = total;
  }
  std::vector<char> host(total, 0);
  char* base = (char*)B->d_plan[grp];
  std::memcpy(host.data(), cs.data(), sizeof(BatchCase) * n);
  const int** offp[5] = {&P.off_cell64, &P.off_face64, &P.off_cell4, &P.off_rec4, &P.off_block};
  for (int k = 0; k < 5; ++k) {
    std::memcpy(host.data() + s_cs + k * s_off, off[k].data(), sizeof(int) * (n + 1));
    *offp[k] = (const int*)(base + s_cs + k * s_off);
  }
  size_t o = s_cs + 5 * s_off;
  const std::vector<std::pair<long long, BatchItem>>* lists[3] = {&mi[0], &mi[1], &ui};
  const BatchItem** dst[3] = {&P.march_items[0], &P.march_items[1], &P.micro_items};
  for (int k = 0; k < 3; ++k) {
    for (size_t e = 0; e < lists[k]->size(); ++e)
      std::memcpy(host.data() + o + e * sizeof(BatchItem), &(*lists[k])[e].second, sizeof(BatchItem));
    *dst[k] = (const BatchItem*)(base + o);
    o += s_it[k];
  }
  P.cases = (const BatchCase*)base;
  if (hipMemcpy(B->d_plan[grp], host.data(), total, hipMemcpyHostToDevice) != hipSuccess)
    return fail(UGKS_E_DEVICE, "upload of the batch plan failed");
  return UGKS_OK;
}

// groups of the batch (one per branch): the cases ordered by tallest block,
// then velocity count, cut into runs of about equal (cell, velocity) pairs,
// so that each group's common launch shapes fit its cases closely
std::vector<std::vector<int>> batch_groups(const ugks_batch* B, int ngroup) {
  const int n = (int)B->ctx.size();
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    const ugks_ctx *a = B->ctx[x], *b = B->ctx[y];
    return a->max_nj != b->max_nj ? a->max_nj < b->max_nj : a->nv < b->nv;
  });
  double total = 0.0;
  for (const ugks_ctx* c : B->ctx) total += (double)c->ncell * c->nv;
  std::vector<std::vector<int>> g(1);
  double acc = 0.0;
  for (int k = 0; k < n; ++k) {
    const ugks_ctx* c = B->ctx[order[k]];
    if (!g.back().empty() && (int)g.size() < ngroup && acc >= total * (double)g.size() / ngroup)
      g.emplace_back();
    g.back().push_back(order[k]);
    acc += (double)c->ncell * c->nv;
  }
  return g;
}

}  // namespace

extern "C" {

int ugks_step_graph(ugks_ctx* c, double dt, int32_t n_inner, void* h, void* b, double* W, const double* Wn,
                    double* q, const void* Sh, const void* Sb, const double* Fn, double* resid, void* stream) {
  if (int rc = check_dev(c, {h, b, W, Wn, q, Sh, Sb, Fn})) return rc;
  if (!(dt > 0) || !std::isfinite(dt)) return fail(UGKS_E_ARG, "dt must be positive");
  if (n_inner < 1) return fail(UGKS_E_ARG, "n_inner must be >= 1");
  std::vector<uint64_t> key = step_key(c, dt, n_inner, {h, b, W, Wn, q, Sh, Sb, Fn, resid});
  if (!c->gexec || key != c->gkey) {
    if (!c->cap) HIPCHK(hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    HIPCHK(hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
    int rc = run_inner(c, dt, n_inner, h, b, W, Wn, q, Sh, Sb, Fn, resid, c->cap, nullptr);
    hipError_t e = hipStreamEndCapture(c->cap, &graph);
    if (!rc && e != hipSuccess) rc = fail(UGKS_E_DEVICE, "stream capture failed");
    if (!rc) rc = graph_to_exec(graph, &c->gexec);
    if (graph) (void)hipGraphDestroy(graph);
    if (rc) { c->gkey.clear(); return rc; }
    c->gkey = key;
  }
  HIPCHK(hipGraphLaunch(c->gexec, (hipStream_t)stream));
  return c->sync_check ? ugks_status(c, stream) : UGKS_OK;
}

int ugks_batch_create(int32_t ncase, ugks_ctx* const* ctxs, ugks_batch** out) {
  if (!out || ncase < 1 || !ctxs) return fail(UGKS_E_ARG, "bad argument");
  *out = nullptr;
  for (int i = 0; i < ncase; ++i) {
    if (!ctxs[i]) return fail(UGKS_E_ARG, "null context");
    if (ctxs[i]->device != ctxs[0]->device) return fail(UGKS_E_ARG, "contexts on different devices");
  }
  auto* B = new ugks_batch;
  B->ctx.assign(ctxs, ctxs + ncase);
  const int ns = std::min(ncase, 4);  // branches: at most the hardware queues of a process
  B->st.assign(ns, nullptr);
  B->ev.assign(ns, nullptr);
  for (int k = 0; k < ns; ++k) {
    if (hipStreamCreateWithFlags(&B->st[k], hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&B->ev[k], hipEventDisableTiming) != hipSuccess) {
      ugks_batch_destroy(B);
      return fail(UGKS_E_DEVICE, "stream or event creation failed");
    }
  }
  *out = B;
  return UGKS_OK;
}

int ugks_batch_destroy(ugks_batch* B) {
  if (!B) return UGKS_OK;
  (void)hipDeviceSynchronize();
  if (B->gexec) (void)hipGraphExecDestroy(B->gexec);
  for (void* p : B->d_plan) if (p) (void)hipFree(p);
  for (auto s : B->st) if (s) (void)hipStreamDestroy(s);
  for (auto e : B->ev) if (e) (void)hipEventDestroy(e);
  delete B;
  return UGKS_OK;
}

int ugks_batch_step(ugks_batch* B, const double* dt, int32_t n_inner, void* const* h, void* const* b,
                    double* const* W, const double* const* Wn, double* const* q, const void* const* Sh,
                    const void* const* Sb, const double* const* Fn, double* const* resid, void* stream) {
  if (!B || !dt || !h || !b || !W || !Wn || !q || !Sh || !Sb || !Fn) return fail(UGKS_E_ARG, "null argument");
  if (n_inner < 1) return fail(UGKS_E_ARG, "n_inner must be >= 1");
  const int n = (int)B->ctx.size();
  std::vector<uint64_t> key;
  for (int i = 0; i < n; ++i) {
    ugks_ctx* c = B->ctx[i];
    double* r = resid ? resid[i] : nullptr;
    if (int rc = check_dev(c, {h[i], b[i], W[i], Wn[i], q[i], Sh[i], Sb[i], Fn[i]})) return rc;
    if (!(dt[i] > 0) || !std::isfinite(dt[i])) return fail(UGKS_E_ARG, "dt must be positive");
    auto k = step_key(c, dt[i], n_inner, {h[i], b[i], W[i], Wn[i], q[i], Sh[i], Sb[i], Fn[i], r});
    key.insert(key.end(), k.begin(), k.end());
  }
  const bool fused = B->mode == 1 && batch_fusable(B);
  key.push_back(fused ? 1 : 0);
  if ((!B->gexec || key != B->gkey) && fused) {
    // one launch per stage for all cases: the plan's tables are rewritten,
    // so no earlier replay may still read them
    HIPCHK(hipDeviceSynchronize());
    const auto groups = batch_groups(B, (int)B->st.size());
    const int ng = (int)groups.size();
    B->plan.resize(ng);
    B->d_plan.resize(ng, nullptr);
    B->plan_bytes.resize(ng, 0);
    for (int k = 0; k < ng; ++k)
      if (int rc = batch_build_plan(B, k, groups[k], dt, h, b, W, Wn, q, Sh, Sb, Fn, resid)) {
        B->gkey.clear();
        return rc;
      }
    hipGraph_t graph = nullptr;
    HIPCHK(hipStreamBeginCapture(B->st[0], hipStreamCaptureModeThreadLocal));
    int rc = UGKS_OK;
    if (hipEventRecord(B->ev[0], B->st[0]) != hipSuccess) rc = fail(UGKS_E_DEVICE, "fork");
    for (int k = 1; k < ng && !rc; ++k)
      if (hipStreamWaitEvent(B->st[k], B->ev[0], 0) != hipSuccess) rc = fail(UGKS_E_DEVICE, "fork");
    for (int k = 0; k < ng && !rc; ++k) launch_batch_inner(B->plan[k], n_inner, B->st[k]);
    if (!rc && hipGetLastError() != hipSuccess) rc = fail(UGKS_E_DEVICE, "batched launch failed");
    for (int k = 1; k < ng && !rc; ++k)
      if (hipEventRecord(B->ev[k], B->st[k]) != hipSuccess || hipStreamWaitEvent(B->st[0], B->ev[k], 0) != hipSuccess)
        rc = fail(UGKS_E_DEVICE, "join");
    hipError_t e = hipStreamEndCapture(B->st[0], &graph);
    if (!rc && e != hipSuccess) rc = fail(UGKS_E_DEVICE, "stream capture failed");
    if (!rc) rc = graph_to_exec(graph, &B->gexec);
    if (graph) (void)hipGraphDestroy(graph);
    if (rc) { B->gkey.clear(); return rc; }
    B->gkey = key;
  }
  if (!B->gexec || key != B->gkey) {
    // one graph: the cases on parallel branches (round robin over the
    // private streams), forked from and joined into the first stream
    const int ns = (int)B->st.size();
    hipGraph_t graph = nullptr;
    HIPCHK(hipStreamBeginCapture(B->st[0], hipStreamCaptureModeThreadLocal));
    int rc = UGKS_OK;
    if (hipEventRecord(B->ev[0], B->st[0]) != hipSuccess) rc = fail(UGKS_E_DEVICE, "fork");
    for (int k = 1; k < ns && !rc; ++k)
      if (hipStreamWaitEvent(B->st[k], B->ev[0], 0) != hipSuccess) rc = fail(UGKS_E_DEVICE, "fork");
    for (int i = 0; i < n && !rc; ++i)
      rc = run_inner(B->ctx[i], dt[i], n_inner, h[i], b[i], W[i], Wn[i], q[i], Sh[i], Sb[i], Fn[i],
                     resid ? resid[i] : nullptr, B->st[i % ns], nullptr);
    for (int k = 1; k < ns && !rc; ++k) {
      if (hipEventRecord(B->ev[k], B->st[k]) != hipSuccess || hipStreamWaitEvent(B->st[0], B->ev[k], 0) != hipSuccess)
        rc = fail(UGKS_E_DEVICE, "join");
    }
    hipError_t e = hipStreamEndCapture(B->st[0], &graph);
    if (!rc && e != hipSuccess) rc = fail(UGKS_E_DEVICE, "stream capture failed");
    if (!rc) rc = graph_to_exec(graph, &B->gexec);
    if (graph) (void)hipGraphDestroy(graph);
    if (rc) { B->gkey.clear(); return rc; }
    B->gkey = key;
  }
  HIPCHK(hipGraphLaunch(B->gexec, (hipStream_t)stream));
  return UGKS_OK;
}

int ugks_batch_set_mode(ugks_batch* B, int32_t mode) {
  if (!B || (mode != 0 && mode != 1)) return fail(UGKS_E_ARG, "mode must be 0 or 1");
  if (mode == 1 && !batch_fusable(B))
    return fail(UGKS_E_UNSUPPORTED, "one launch per stage needs 2D cases of one storage type");
  if (B->mode != mode) {
    B->mode = mode;
    B->gkey.clear();
  }
  return UGKS_OK;
}

int ugks_batch_get_mode(const ugks_batch* B, int32_t* mode) {
  if (!B || !mode) return fail(UGKS_E_ARG, "null argument");
  *mode = (B->mode == 1 && batch_fusable(B)) ? 1 : 0;
  return UGKS_OK;
}

int ugks_set_tuning(ugks_ctx* c, int32_t kc_max, int32_t rg_eq, int32_t rg_flux) {
  if (!c) return fail(UGKS_E_ARG, "null context");
  if ((kc_max != 16 && kc_max != 8 && kc_max != 4) || (rg_eq != 10 && rg_eq != 8 && rg_eq != 6) ||
      (rg_flux != 10 && rg_flux != 8 && rg_flux != 6))
    return fail(UGKS_E_ARG, "kc_max must be 16, 8 or 4, rg_eq and rg_flux 10, 8 or 6");
  c->dev.kc_max = kc_max;
  c->dev.rg_eq = rg_eq;
  c->dev.rg_flux = rg_flux;
  ++c->version;
  return UGKS_OK;
}

int ugks_get_tuning(const ugks_ctx* c, int32_t* kc_max, int32_t* rg_eq, int32_t* rg_flux) {
  if (!c) return fail(UGKS_E_ARG, "null context");
  if (kc_max) *kc_max = c->dev.kc_max;
  if (rg_eq) *rg_eq = c->dev.rg_eq;
  if (rg_flux) *rg_flux = c->dev.rg_flux;
  return UGKS_OK;
}

int ugks_micro_shape(const ugks_ctx* c, int32_t* kc, int32_t* rows, int32_t* depth, int32_t* fused) {
  if (!c) return fail(UGKS_E_ARG, "null context");
  int k, r, p, f;
  micro_launch_shape(c->dim, c->prec, c->max_ni, c->max_nj, c->any_pj, c->dev.kc_max, k, r, p, f);
  if (kc) *kc = k;
  if (rows) *rows = r;
  if (depth) *depth = p;
  if (fused) *fused = f;
  return UGKS_OK;
}

int ugks_autotune(ugks_ctx* c, double dt, int32_t n_inner, const void* h, const void* b, const double* W,
                  const double* Wn, const double* q, const void* Sh, const void* Sb, const double* Fn,
                  int32_t* choice, double* best_ms, void* stream) {
  if (int rc = check_dev(c, {h, b, W, Wn, q, Sh, Sb, Fn})) return rc;
  if (!(dt > 0) || !std::isfinite(dt)) return fail(UGKS_E_ARG, "dt must be positive");
  if (n_inner < 1) return fail(UGKS_E_ARG, "n_inner must be >= 1");
  hipStream_t st = (hipStream_t)stream;
  const size_t fb = (size_t)c->ncell * c->nv * (c->prec == UGKS_F64 ? 8 : 4);
  const size_t wb = sizeof(double) * c->nw * (size_t)c->ncell, qb = sizeof(double) * c->dim * (size_t)c->ncell;
  void *th = nullptr, *tb = nullptr, *tW = nullptr, *tq = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = UGKS_OK;
  // state copies: in the adjoint workspace when the context has one (its
  // first buffers are [ncell][nv] doubles, [ncell][nw] and [ncell][dim]),
  // else allocated for the call
  const bool in_adj = !c->adj.empty();
  if (in_adj) {
    th = c->adj[0]; tb = c->adj[1]; tW = c->adj[14]; tq = c->adj[16];
  } else if (hipMalloc(&th, fb) != hipSuccess || hipMalloc(&tb, fb) != hipSuccess ||
             hipMalloc(&tW, wb) != hipSuccess || hipMalloc(&tq, qb) != hipSuccess) {
    rc = fail(UGKS_E_DEVICE, "autotune scratch");
  }
  if (!rc && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
    rc = fail(UGKS_E_DEVICE, "autotune events");
  const Dev saved = c->dev;
  double best = 1e300;
  int bk = saved.kc_max, be = saved.rg_eq, bf = saved.rg_flux;
  // one run from the same inputs (copies; the caller's arrays are not
  // written) with shapes (kc, re, rf); its time in ms, or < 0 when skipped
  auto trial = [&](int kc, int re, int rf) -> double {
    if (rc) return -1.0;
    if (micro_lds(c->dim, c->max_ni, c->max_nj, c->any_pj, kc) > 160 * 1024) return -1.0;
    c->dev.kc_max = kc; c->dev.rg_eq = re; c->dev.rg_flux = rf;
    if (hipMemcpyAsync(th, h, fb, hipMemcpyDeviceToDevice, st) != hipSuccess ||
        hipMemcpyAsync(tb, b, fb, hipMemcpyDeviceToDevice, st) != hipSuccess ||
        hipMemcpyAsync(tW, W, wb, hipMemcpyDeviceToDevice, st) != hipSuccess ||
        hipMemcpyAsync(tq, q, qb, hipMemcpyDeviceToDevice, st) != hipSuccess ||
        hipEventRecord(e0, st) != hipSuccess) { rc = fail(UGKS_E_DEVICE, "autotune copy"); return -1.0; }
    rc = run_inner(c, dt, n_inner, th, tb, (double*)tW, Wn, (double*)tq, Sh, Sb, Fn, nullptr, st, nullptr);
    if (rc) return -1.0;
    float ms = 0.f;
    if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { rc = fail(UGKS_E_DEVICE, "autotune timing"); return -1.0; }
    return ms;
  };
  // the three shapes act on different kernels (micro sweep, face-moment
  // march, flux march): one coordinate at a time, the others at their best
  auto consider = [&](int kc, int re, int rf) {
    const double ms = trial(kc, re, rf);
    if (ms >= 0.0 && ms < best) { best = ms; bk = kc; be = re; bf = rf; }
  };
  consider(16, 8, 8);
  consider(8, 8, 8);
  consider(4, 8, 8);
  const int kc1 = bk;
  for (int re : {10, 6}) consider(kc1, re, 8);
  const int re1 = be;
  for (int rf : {10, 6}) consider(kc1, re1, rf);
  c->dev = saved;
  if (!rc) {
    c->dev.kc_max = bk; c->dev.rg_eq = be; c->dev.rg_flux = bf;
    ++c->version;
    if (choice) { choice[0] = bk; choice[1] = be; choice[2] = bf; }
    if (best_ms) *best_ms = best / n_inner;
  }
  if (!in_adj)
    for (void* p : {th, tb, tW, tq}) if (p) (void)hipFree(p);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  return rc;
}


// ---------------------------------------------------------------------------
// reverse mode (adjoint) of Steps 1-2, of the pseudo-iteration and of the flux
// ---------------------------------------------------------------------------
}  // extern "C"

namespace {

enum AdjBuf {
  // [ncell][nv]
  A_H0, A_B0, A_H1, A_B1, A_XBH, A_XBB, A_YH, A_YB, A_RH, A_RB, A_DBH, A_DBB, A_HB, A_BB,
  // [ncell][nw], [ncell][dim]
  A_W0, A_W1, A_Q0, A_Q1, A_WPB, A_DWB, A_ABAR, A_BBAR, A_DWSB, A_RBAR, A_WB, A_QB,
  // others
  A_DGB, A_GWB, A_GAMB, A_FB, A_FBAR,
  // [ncell][4][2]: face-velocity bars of the micro coefficients per cell side
  A_SLOT,
  // int32 items of the scatter colourings: every face, every cell, and up
  // to 2 ncell donor rows (receptor rows and refill rows are cells)
  A_ORD,
  // [kFaceBlocks][6][nv]: per-velocity bars staged by the face reverse
  A_FSC, A_NBUF
};

std::vector<size_t> adjoint_counts(const Sizes& z) {
  const size_t N = (size_t)z.ncell * z.nv, NW = (size_t)z.ncell * z.nw, NQ = (size_t)z.ncell * z.dim;
  std::vector<size_t> out(A_NBUF);
  for (int i = 0; i < A_NBUF; ++i) {
    size_t n;
    if (i <= A_BB) n = N;
    else if (i == A_Q0 || i == A_Q1 || i == A_QB) n = NQ;
    else if (i <= A_WB) n = NW;
    else if (i == A_DGB) n = z.ncell;
    else if (i == A_GWB) n = 8 * (size_t)z.ncell;
    else if (i == A_GAMB) n = z.nface;
    else if (i == A_FB) n = (size_t)z.nface * z.nw;
    else if (i == A_SLOT) n = 8 * (size_t)z.ncell;
    else if (i == A_ORD) n = ((size_t)z.nface + 3 * (size_t)z.ncell + 1) / 2;
    else if (i == A_FSC) n = (size_t)kFaceBlocks * 6 * z.nv;
    else n = (size_t)z.nface * 5;
    out[i] = n;
  }
  return out;
}

// the adjoint workspace: the caller's (carved at creation) or one
// allocation on first use
int adj_alloc(ugks_ctx* c) {
  if (!c->adj.empty()) return UGKS_OK;
  const Sizes z = sizes_of(c);
  void* base = nullptr;
  if (hipMalloc(&base, adjoint_bytes(z)) != hipSuccess) return fail(UGKS_E_DEVICE, "adjoint workspace allocation");
  carve_adjoint(c, z, (char*)base);
  c->own_adj = true;
  return UGKS_OK;
}

double* A(ugks_ctx* c, int i) { return (double*)c->adj[i]; }

// Greedy colouring of items by their write sets: the items, in the order
// given, each take the lowest colour that no earlier item sharing a
// resource holds.  `res(id, out)` lists an item's resources (ids below
// nres).  Appends the item ids sorted by colour (in the given order within
// a colour) to `order` and returns the colour offsets relative to its first
// entry.
template <typename R>
int colour_items(const std::vector<int>& ids, int nres, R res, std::vector<int>& order, std::vector<int>& off) {
  constexpr int kW = 4;  // up to 256 colours
  const int n = (int)ids.size();
  std::vector<uint64_t> used((size_t)nres * kW, 0);
  std::vector<int> col(n), set;
  int ncol = 0;
  for (int i = 0; i < n; ++i) {
    set.clear();
    res(ids[i], set);
    uint64_t busy[kW] = {0, 0, 0, 0};
    for (int r : set)
      for (int w = 0; w < kW; ++w) busy[w] |= used[(size_t)r * kW + w];
    int k = 0;
    while (k < 64 * kW && ((busy[k >> 6] >> (k & 63)) & 1)) ++k;
    if (k == 64 * kW) return fail(UGKS_E_UNSUPPORTED, "scatter colouring needs more than 256 colours");
    col[i] = k;
    ncol = std::max(ncol, k + 1);
    for (int r : set) used[(size_t)r * kW + (k >> 6)] |= uint64_t(1) << (k & 63);
  }
  off.assign(ncol + 1, 0);
  for (int i = 0; i < n; ++i) ++off[col[i] + 1];
  for (int k = 0; k < ncol; ++k) off[k + 1] += off[k];
  const size_t base = order.size();
  order.resize(base + n);
  std::vector<int> pos(off.begin(), off.end() - 1);
  for (int i = 0; i < n; ++i) order[base + pos[col[i]]++] = ids[i];
  return UGKS_OK;
}

std::vector<int> iota_ids(int n) {
  std::vector<int> v(std::max(n, 0));
  for (int i = 0; i < n; ++i) v[i] = i;
  return v;
}

// the colourings of the reverse-mode scatters for the current tables
int adj_orders(ugks_ctx* c) {
  if (c->ord_version == (long long)c->version) return UGKS_OK;
  const int nc = c->ncell;
  auto cell_nb = [&](int x, std::vector<int>& out) {
    out.push_back(x);
    for (int s = 0; s < 4; ++s)
      if (c->nb[4 * (size_t)x + s] >= 0) out.push_back(c->nb[4 * (size_t)x + s]);
  };
  std::vector<int> order, inner_faces, wall_faces;
  for (int f = 0; f < c->nface; ++f) {
    const bool wall = c->fcell[2 * (size_t)f] == kNbWall || c->fcell[2 * (size_t)f + 1] == kNbWall;
    (wall ? wall_faces : inner_faces).push_back(f);
  }
  // faces: the cells whose bars the face reverse (reconstruction of either
  // side, wall incident state, spectral radius) can update
  auto face_res = [&](int f, std::vector<int>& out) {
    const int L = c->fcell[2 * (size_t)f], R = c->fcell[2 * (size_t)f + 1];
    if (L == kNbWall || R == kNbWall) {
      const int x = (L == kNbWall) ? R : L;
      if (x >= 0) cell_nb(x, out);
      return;
    }
    const int inner = (L >= 0) ? L : R;
    for (int x : {L, R}) {
      if (x >= 0) cell_nb(x, out);
      else if (inner >= 0) out.push_back(inner);
    }
  };
  int rc = colour_items(inner_faces, nc, face_res, order, c->ord_off[0]);
  // cells: the limited W gradients reversed write c and its neighbours
  if (!rc) rc = colour_items(iota_ids(nc), nc, cell_nb, order, c->ord_off[1]);
  // donor rows: the target and its donors, receptor rows and refill rows
  // apart (they are reversed by separate launches)
  const int nrow = (int)c->h_rec.size();
  for (int part = 0; part < 2 && !rc; ++part) {
    const int r0 = part ? c->nrec : 0, n = part ? nrow - c->nrec : c->nrec;
    rc = colour_items(iota_ids(n), nc, [&](int r, std::vector<int>& out) {
      out.push_back(c->h_rec[r0 + r]);
      for (int p = c->h_ptr[r0 + r]; p < c->h_ptr[r0 + r + 1]; ++p) out.push_back(c->h_don[p]);
    }, order, c->ord_off[2 + part]);
  }
  if (!rc) rc = colour_items(wall_faces, nc, face_res, order, c->ord_off[4]);
  if (rc) return rc;
  if (order.size() > (size_t)c->nface + 3 * (size_t)c->ncell) return fail(UGKS_E_SHAPE, "donor table larger than 2 ncell rows");
  // earlier reverse calls, on any stream, may still read the old orders
  HIPCHK(hipDeviceSynchronize());
  HIPCHK(hipMemcpy(A(c, A_ORD), order.data(), sizeof(int) * order.size(), hipMemcpyHostToDevice));
  c->ord_version = (long long)c->version;
  return UGKS_OK;
}

// colouring `k` (0 faces other than wall faces, 1 cells, 2 receptor rows,
// 3 refill rows, 4 wall faces) as a launch order
Order order_of(ugks_ctx* c, int k) {
  size_t base = 0;
  for (int i = 0; i < k; ++i) base += c->ord_off[i].back();
  Order o;
  o.items = (const int*)A(c, A_ORD) + base;
  o.off = c->ord_off[k].data();
  o.ncolour = (int)c->ord_off[k].size() - 1;
  return o;
}

int adj_check(ugks_ctx* c) {
  if (!c) return fail(UGKS_E_ARG, "null context");
  if (c->prec != UGKS_F64) return fail(UGKS_E_UNSUPPORTED, "the adjoint needs FP64 storage");
  if (c->dim != 2) return fail(UGKS_E_UNSUPPORTED, "the adjoint is built for 2D cases");
  if (int rc = adj_alloc(c)) return rc;
  return adj_orders(c);
}

int dcopy(void* dst, const void* src, size_t n, hipStream_t st) {
  HIPCHK(hipMemcpyAsync(dst, src, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
  return UGKS_OK;
}

int dzero(void* dst, size_t n, hipStream_t st) {
  HIPCHK(hipMemsetAsync(dst, 0, sizeof(double) * n, st));
  return UGKS_OK;
}

// copy of a cotangent argument, or zeros when it is NULL
int dcopy_or_zero(void* dst, const void* src, size_t n, hipStream_t st) {
  return src ? dcopy(dst, src, n, st) : dzero(dst, n, st);
}

// the flux reverse at (H0, B0, W0, Q0) with divergence bars A_DBH/A_DBB and
// face-flux bar A_FB: accumulates into A_HB, A_BB, A_WB, A_QB, A_FBAR
// (s_gW and s_rec must hold the forward gradients of W0 and face records)
int flux_reverse(ugks_ctx* c, hipStream_t st) {
  if (int rc = dzero(A(c, A_GWB), 8 * (size_t)c->ncell, st)) return rc;
  adj_flux(c->dev, order_of(c, 0), order_of(c, 4), order_of(c, 1), c->dts, A(c, A_H0), A(c, A_B0), A(c, A_W0), A(c, A_Q0),
           (const double*)c->s_gW,
           (const double*)c->s_rec, A(c, A_DBH),
           A(c, A_DBB), A(c, A_FB), A(c, A_HB), A(c, A_BB), A(c, A_WB), A(c, A_QB), A(c, A_GWB), A(c, A_FBAR),
           A(c, A_FSC), st);
  HIPCHK(hipGetLastError());
  return UGKS_OK;
}

int interp_rows(ugks_ctx* c, int r0, int nrow, double* h, double* b, double* W, double* q, hipStream_t st) {
  if (nrow <= 0) return UGKS_OK;
  launch_interp(c->dev, c->prec, nrow, (const int*)c->d_rec + r0, (const int*)c->d_ptr + r0, (const int*)c->d_don,
                (const double*)c->d_w, h, b, W, q, st);
  HIPCHK(hipGetLastError());
  return UGKS_OK;
}

// rows r0 .. r0 + nrow - 1 reversed: the receptor rows (refill false, r0 =
// 0) or the refill rows after them
int interp_rows_rev(ugks_ctx* c, bool refill, int r0, int nrow, hipStream_t st) {
  if (nrow <= 0) return UGKS_OK;
  adj_interp(c->dev, order_of(c, refill ? 3 : 2), (const int*)c->d_rec + r0, (const int*)c->d_ptr + r0, (const int*)c->d_don,
             (const double*)c->d_w, A(c, A_HB), A(c, A_BB), A(c, A_WB), A(c, A_QB), st);
  HIPCHK(hipGetLastError());
  return UGKS_OK;
}

// load the state into the workspace (H0.. = copies)
int load_state(ugks_ctx* c, const void* h, const void* b, const double* W, const double* q, hipStream_t st) {
  const size_t N = (size_t)c->ncell * c->nv;
  int rc = dcopy(A(c, A_H0), h, N, st);
  if (!rc) rc = dcopy(A(c, A_B0), b, N, st);
  if (!rc) rc = dcopy(A(c, A_W0), W, (size_t)c->ncell * c->nw, st);
  if (!rc) rc = dcopy(A(c, A_Q0), q, (size_t)c->ncell * c->dim, st);
  return rc;
}

int store_bars(ugks_ctx* c, double* hb, double* bb, double* Wb, double* qb, double* faceb, hipStream_t st) {
  const size_t N = (size_t)c->ncell * c->nv;
  int rc = UGKS_OK;
  if (!rc && hb) rc = dcopy(hb, A(c, A_HB), N, st);
  if (!rc && bb) rc = dcopy(bb, A(c, A_BB), N, st);
  if (!rc && Wb) rc = dcopy(Wb, A(c, A_WB), (size_t)c->ncell * c->nw, st);
  if (!rc && qb) rc = dcopy(qb, A(c, A_QB), (size_t)c->ncell * c->dim, st);
  if (!rc && faceb) rc = dcopy(faceb, A(c, A_FBAR), 5 * (size_t)c->nface, st);
  return rc;
}

}  // namespace

extern "C" {

int ugks_flux_adjoint(ugks_ctx* c, const void* h, const void* b, const double* W, const double* q,
                      const double* Dh_bar, const double* Db_bar, const double* F_bar, double* h_bar, double* b_bar,
                      double* W_bar, double* q_bar, double* face_bar, void* stream) {
  if (int rc = check_dev(c, {h, b, W, q, h_bar, b_bar, W_bar, q_bar})) return rc;
  if (int rc = adj_check(c)) return rc;
  hipStream_t st = (hipStream_t)stream;
  const size_t N = (size_t)c->ncell * c->nv;
  int rc = load_state(c, h, b, W, q, st);
  // forward: the W gradients (the divergence and face fluxes land in scratch)
  if (!rc) rc = dzero(c->s_F, (size_t)c->nw * c->nface, st);
  if (rc) return rc;
  launch_flux(c->dev, c->prec, (const int*)c->d_binfo, c->max_nj, c->dts, A(c, A_H0), A(c, A_B0), A(c, A_W0),
              A(c, A_Q0), (double*)c->s_gW, (double*)c->s_rec, (double*)c->s_part, c->s_Dh, c->s_Db,
              (double*)c->s_F, nullptr, st);
  HIPCHK(hipGetLastError());
  rc = dcopy_or_zero(A(c, A_DBH), Dh_bar, N, st);
  if (!rc) rc = dcopy_or_zero(A(c, A_DBB), Db_bar, N, st);
  if (!rc) rc = dcopy_or_zero(A(c, A_FB), F_bar, (size_t)c->nface * c->nw, st);
  for (int i : {A_HB, A_BB}) if (!rc) rc = dzero(A(c, i), N, st);
  if (!rc) rc = dzero(A(c, A_WB), (size_t)c->ncell * c->nw, st);
  if (!rc) rc = dzero(A(c, A_QB), (size_t)c->ncell * c->dim, st);
  if (!rc) rc = dzero(A(c, A_FBAR), 5 * (size_t)c->nface, st);
  if (!rc) rc = flux_reverse(c, st);
  if (!rc) rc = store_bars(c, h_bar, b_bar, W_bar, q_bar, face_bar, st);
  return rc;
}

int ugks_step_adjoint(ugks_ctx* c, double dt, const void* h, const void* b, const double* W, const double* Wn,
                      const double* q, const void* Sh, const void* Sb, const double* Fn, const double* h1_bar,
                      const double* b1_bar, const double* W1_bar, const double* q1_bar, const double* F_bar,
                      double* h_bar, double* b_bar, double* W_bar, double* Wn_bar, double* q_bar, double* Sh_bar,
                      double* Sb_bar, double* Fn_bar, double* face_bar, void* stream) {
  if (int rc = check_dev(c, {h, b, W, Wn, q, Sh, Sb, Fn, h_bar, b_bar, W_bar, Wn_bar, q_bar, Sh_bar, Sb_bar,
                             Fn_bar}))
    return rc;
  if (!(dt > 0) || !std::isfinite(dt)) return fail(UGKS_E_ARG, "dt must be positive");
  if (int rc = adj_check(c)) return rc;
  hipStream_t st = (hipStream_t)stream;
  const Dev& g = c->dev;
  const size_t N = (size_t)c->ncell * c->nv, NW = (size_t)c->ncell * c->nw, NQ = (size_t)c->ncell * c->dim;
  const int nblock = (int)c->blk.size();
  // forward recomputation: the interpolated input state (H0..) and one
  // pseudo-iteration from it (H1..); the solver's scratch keeps the
  // intermediates (W gradients, Gamma, dW*, dW, W~ and its record, dF*)
  int rc = load_state(c, h, b, W, q, st);
  if (!rc) rc = interp_rows(c, 0, c->nrec, A(c, A_H0), A(c, A_B0), A(c, A_W0), A(c, A_Q0), st);
  if (!rc) rc = dcopy(A(c, A_H1), A(c, A_H0), N, st);
  if (!rc) rc = dcopy(A(c, A_B1), A(c, A_B0), N, st);
  if (!rc) rc = dcopy(A(c, A_W1), A(c, A_W0), NW, st);
  if (!rc) rc = dcopy(A(c, A_Q1), A(c, A_Q0), NQ, st);
  if (!rc) rc = run_inner(c, dt, 1, A(c, A_H1), A(c, A_B1), A(c, A_W1), Wn, A(c, A_Q1), Sh, Sb, Fn, nullptr, st,
                          nullptr);
  if (rc) return rc;
  // Step 7 and the new heat flux
  rc = dcopy_or_zero(A(c, A_XBH), h1_bar, N, st);
  if (!rc) rc = dcopy_or_zero(A(c, A_XBB), b1_bar, N, st);
  if (!rc) rc = dcopy_or_zero(A(c, A_RBAR), W1_bar, NW, st);  // staging of W' bar
  if (!rc) rc = dcopy_or_zero(A(c, A_QB), q1_bar, NQ, st);    // staging of q' bar
  if (rc) return rc;
  adj_step7(g, A(c, A_H1), A(c, A_B1), A(c, A_W1), (const double*)c->s_Wp, A(c, A_RBAR), A(c, A_QB), A(c, A_XBH),
            A(c, A_XBB), A(c, A_WPB), st);
  HIPCHK(hipGetLastError());
  // micro LU-SGS (Steps 5-6); dF* is in s_Dh, s_Db
  rc = dzero(A(c, A_FBAR), 5 * (size_t)c->nface, st);
  if (rc) return rc;
  adj_micro(g, (const int*)c->d_binfo, nblock, dt, (const double*)c->s_crec, (const double*)c->s_Wp, A(c, A_H0),
            A(c, A_B0), A(c, A_H1), A(c, A_B1), (const double*)c->s_Dh, (const double*)c->s_Db, A(c, A_XBH),
            A(c, A_XBB), A(c, A_YH), A(c, A_YB), A(c, A_RH), A(c, A_RB), A(c, A_HB), A(c, A_BB), Sh_bar, Sb_bar,
            A(c, A_DBH), A(c, A_DBB), A(c, A_WPB), A(c, A_SLOT), A(c, A_FBAR), st);
  HIPCHK(hipGetLastError());
  // macro LU-SGS (Step 4)
  rc = dzero(A(c, A_WB), NW, st);
  if (!rc) rc = dzero(Wn_bar, NW, st);
  if (!rc) rc = dzero(Fn_bar, (size_t)c->nface * c->nw, st);
  if (!rc) rc = dcopy_or_zero(A(c, A_FB), F_bar, (size_t)c->nface * c->nw, st);
  if (!rc) rc = dzero(A(c, A_DGB), c->ncell, st);
  if (!rc) rc = dzero(A(c, A_GAMB), c->nface, st);
  if (rc) return rc;
  adj_macro(g, order_of(c, 0), order_of(c, 4), (const int*)c->d_binfo, nblock, dt, A(c, A_W0), (const double*)c->s_dWs, (const double*)c->s_dW,
            (const double*)c->s_gam, A(c, A_WPB), A(c, A_DWB), A(c, A_ABAR), A(c, A_BBAR), A(c, A_DWSB),
            A(c, A_RBAR), A(c, A_DGB), A(c, A_GAMB), A(c, A_WB), Wn_bar, A(c, A_FB), Fn_bar, A(c, A_FBAR), st);
  HIPCHK(hipGetLastError());
  // flux (Step 3) at the interpolated state, then the interpolation
  rc = dzero(A(c, A_QB), NQ, st);
  if (!rc) rc = flux_reverse(c, st);
  if (!rc) rc = interp_rows_rev(c, false, 0, c->nrec, st);
  if (!rc) rc = store_bars(c, h_bar, b_bar, W_bar, q_bar, face_bar, st);
  return rc;
}

int ugks_begin_step_adjoint(ugks_ctx* c, double dt, const void* h, const void* b, const double* W, const double* q,
                            int32_t refill, const double* h1_bar, const double* b1_bar, const double* W1_bar,
                            const double* q1_bar, const double* Sh_bar, const double* Sb_bar, const double* Fn_bar,
                            double* h_bar, double* b_bar, double* W_bar, double* q_bar, double* face_bar,
                            void* stream) {
  if (int rc = check_dev(c, {h, b, W, q, Sh_bar, Sb_bar, h_bar, b_bar, W_bar, q_bar})) return rc;
  if (!(dt > 0) || !std::isfinite(dt)) return fail(UGKS_E_ARG, "dt must be positive");
  if (int rc = adj_check(c)) return rc;
  hipStream_t st = (hipStream_t)stream;
  const size_t N = (size_t)c->ncell * c->nv, NW = (size_t)c->ncell * c->nw, NQ = (size_t)c->ncell * c->dim;
  const int nref = refill ? (int)c->h_rec.size() - c->nrec : 0;
  // forward: refills, receptors, the W gradients and the cell records
  int rc = load_state(c, h, b, W, q, st);
  if (!rc) rc = interp_rows(c, c->nrec, nref, A(c, A_H0), A(c, A_B0), A(c, A_W0), A(c, A_Q0), st);
  if (!rc) rc = interp_rows(c, 0, c->nrec, A(c, A_H0), A(c, A_B0), A(c, A_W0), A(c, A_Q0), st);
  if (!rc) rc = dzero(A(c, A_FB), (size_t)c->nface * c->nw, st);
  if (rc) return rc;
  launch_flux(c->dev, c->prec, (const int*)c->d_binfo, c->max_nj, c->dts, A(c, A_H0), A(c, A_B0), A(c, A_W0),
              A(c, A_Q0), (double*)c->s_gW, (double*)c->s_rec, (double*)c->s_part, A(c, A_DBH), A(c, A_DBB),
              A(c, A_FB), nullptr, st);
  launch_cellrec(c->dev, dt, A(c, A_W0), A(c, A_Q0), nullptr, (double*)c->s_crec, st);
  HIPCHK(hipGetLastError());
  // reverse
  rc = dcopy_or_zero(A(c, A_HB), h1_bar, N, st);
  if (!rc) rc = dcopy_or_zero(A(c, A_BB), b1_bar, N, st);
  if (!rc) rc = dcopy_or_zero(A(c, A_WB), W1_bar, NW, st);
  if (!rc) rc = dcopy_or_zero(A(c, A_QB), q1_bar, NQ, st);
  if (!rc) rc = dcopy_or_zero(A(c, A_FB), Fn_bar, (size_t)c->nface * c->nw, st);
  if (!rc) rc = dzero(A(c, A_FBAR), 5 * (size_t)c->nface, st);
  if (rc) return rc;
  adj_source(c->dev, dt, (const double*)c->s_crec, A(c, A_W0), A(c, A_H0), A(c, A_B0), Sh_bar, Sb_bar, A(c, A_HB),
             A(c, A_BB), A(c, A_DBH), A(c, A_DBB), A(c, A_WB), A(c, A_QB), st);
  HIPCHK(hipGetLastError());
  rc = flux_reverse(c, st);
  if (!rc) rc = interp_rows_rev(c, false, 0, c->nrec, st);
  if (!rc) rc = interp_rows_rev(c, true, c->nrec, nref, st);
  if (!rc) rc = store_bars(c, h_bar, b_bar, W_bar, q_bar, face_bar, st);
  return rc;
}


// ---------------------------------------------------------------------------
// status of the device-side checks, wall loads, parameter cotangents
// ---------------------------------------------------------------------------
int ugks_status(ugks_ctx* c, void* stream) {
  if (!c) return fail(UGKS_E_ARG, "null context");
  HIPCHK(hipStreamSynchronize((hipStream_t)stream));
  unsigned st = 0;
  HIPCHK(hipMemcpy(&st, c->d_status, sizeof st, hipMemcpyDeviceToHost));
  if (st == 0) return UGKS_OK;
  const unsigned zero = 0;
  HIPCHK(hipMemcpy(c->d_status, &zero, sizeof zero, hipMemcpyHostToDevice));
  if (st & kStatusWait)
    return fail(UGKS_E_DEVICE, "a micro sweep's wait for its neighbour wavefronts ran out; its results are not valid");
  return fail(UGKS_E_NONPHYS, "Step 7 produced a non-positive density or temperature, or a non-finite state");
}

int ugks_set_checks(ugks_ctx* c, int32_t sync, int32_t wait_limit) {
  if (!c) return fail(UGKS_E_ARG, "null context");
  c->sync_check = sync ? 1 : 0;
  const int lim = (wait_limit < 0) ? (1 << 20) : wait_limit;
  if (lim != c->dev.micro_spin) {
    c->dev.micro_spin = lim;
    ++c->version;  // captured graphs hold the kernels' arguments
  }
  return UGKS_OK;
}

int ugks_wall_loads(ugks_ctx* c, const double* F, double* face_loads, double* side_loads, void* stream) {
  if (int rc = check_dev(c, {F})) return rc;
  launch_wall_loads(c->dev, 4 * (int)c->blk.size(), (const int*)c->d_wptr, (const double*)c->d_wtab, F, face_loads,
                    side_loads, (hipStream_t)stream);
  HIPCHK(hipGetLastError());
  return UGKS_OK;
}

int ugks_wall_loads_adjoint(ugks_ctx* c, const double* face_loads_bar, const double* side_loads_bar, double* F_bar,
                            void* stream) {
  if (int rc = check_dev(c, {F_bar})) return rc;
  launch_wall_loads_adj(c->dev, 4 * (int)c->blk.size(), (const int*)c->d_wptr, (const double*)c->d_wtab,
                        face_loads_bar, side_loads_bar, F_bar, (hipStream_t)stream);
  HIPCHK(hipGetLastError());
  return UGKS_OK;
}

int ugks_param_bars(ugks_ctx* c, const double* face_bar, double* U_bar, double* rtw_bar, void* stream) {
  if (int rc = check_dev(c, {face_bar, U_bar, rtw_bar})) return rc;
  launch_param_bars((int)c->blk.size(), (const int*)c->d_bface, (const int*)c->d_wptr, (const double*)c->d_wtab,
                    face_bar, U_bar, rtw_bar, (hipStream_t)stream);
  HIPCHK(hipGetLastError());
  return UGKS_OK;
}

int ugks_newton_euler(ugks_ctx* c, int32_t blk, const double* body, double dt, const double* F, double* pose,
                      void* stream) {
  if (int rc = check_dev(c, {F})) return rc;
  if (!body || !pose) return fail(UGKS_E_ARG, "null host array");
  if (c->dim != 2) return fail(UGKS_E_UNSUPPORTED, "rigid-body motion is built for 2D cases");
  if (blk < 0 || blk >= (int)c->blk.size()) return fail(UGKS_E_ARG, "bad block");
  if (!(body[0] > 0) || !(body[1] > 0) || !std::isfinite(body[0]) || !std::isfinite(body[1]))
    return fail(UGKS_E_ARG, "mass and moment of inertia must be positive");
  if (!(dt > 0) || !std::isfinite(dt)) return fail(UGKS_E_ARG, "dt must be positive");
  hipStream_t st = (hipStream_t)stream;
  launch_wall_loads(c->dev, 4 * (int)c->blk.size(), (const int*)c->d_wptr, (const double*)c->d_wtab, F, nullptr,
                    (double*)c->d_side, st);
  HIPCHK(hipGetLastError());
  std::vector<double> side(16 * c->blk.size());
  HIPCHK(hipMemcpyAsync(side.data(), c->d_side, sizeof(double) * side.size(), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  // force and moment on the body: its walls' loads plus the external load;
  // velocities by an explicit step, the pose by the trapezoidal rule (exact
  // for constant loads)
  double fx = body[2], fy = body[3], mz = body[4];
  for (int sd = 0; sd < 4; ++sd) {
    if (c->blk[blk].bc[sd] != UGKS_BC_WALL) continue;
    fx += side[16 * (size_t)blk + 4 * sd + 0];
    fy += side[16 * (size_t)blk + 4 * sd + 1];
    mz += side[16 * (size_t)blk + 4 * sd + 2];
  }
  const double ux = pose[3] + dt * fx / body[0];
  const double uy = pose[4] + dt * fy / body[0];
  const double om = pose[5] + dt * mz / body[1];
  pose[0] += 0.5 * dt * (pose[3] + ux);
  pose[1] += 0.5 * dt * (pose[4] + uy);
  pose[2] += 0.5 * dt * (pose[5] + om);
  pose[3] = ux; pose[4] = uy; pose[5] = om;
  return UGKS_OK;
}

}  // extern "C"
