// Host overset assembly of libugks (Sec. 3.1, Sec. 3.2).
//
// Each block is one grid zone.  Integer results (node and cell classes,
// receptors, donors) are decided by these geometric predicates, evaluated
// in plain double arithmetic without contraction (this file is compiled
// with -ffp-contract=off), so that they are reproducible bit for bit:
//   point in quad   every edge cross product (q[k+1]-q[k]) x (p-q[k]) of one
//                   sign or zero; edges and corners count as inside;
//   wall distance   squared distance to the nearest wall segment of a zone,
//                   +inf for a zone without walls;
//   inside a body   crossing number (half-open in y) against each closed wall
//                   outline (a wall side of a block periodic along it) of the
//                   other zones.
// A node of zone A is inactive inside another zone's body, or where another
// zone B has a cell containing it (the lowest such cell, at least overlap+3
// cell layers inside B's overset sides) and a nearer wall (ties: the higher
// zone).  Cells are field (all nodes active), hole (none) or boundary;
// receptors are the boundary cells, one buffer layer of field cells beside
// boundary or hole cells, and `overlap` layers beside overset sides.  The
// donor of a receptor is the field cell of another zone containing its
// centroid (lowest zone, then lowest cell).  Weights: inverse distance
// squared over the donor and its field index neighbours (exact copy at zero
// distance), or bilinear over the quad of donor-grid centroids around the
// receptor (three Newton steps from the quad middle; inverse distance where
// no such quad of field cells contains the point).
//
// Point location uses a uniform bucket grid per zone (candidates in cell
// order), which only prunes the search: the first containing cell in cell
// order is the same as in an exhaustive scan.
#include "ugks_overset.h"

#include <algorithm>
#include <cmath>
#include <limits>
#include <thread>

#include "ugks.h"

namespace ugks {
namespace {

constexpr int kBig = 1 << 30;

struct Zone {
  int ni = 0, nj = 0, cell0 = 0, bc[4] = {0, 0, 0, 0};
  size_t node0 = 0;
  // bucket grid over the zone's bounding box
  double x0 = 0, y0 = 0, x1 = 0, y1 = 0, dx = 1, dy = 1, eps = 0;
  int nbx = 1, nby = 1;
  std::vector<int> start, items;
};

struct Ctx {
  const OversetInput& in;
  std::vector<Zone> z;
  explicit Ctx(const OversetInput& i) : in(i) {}
  double X(int b, int i, int j) const { return (*in.xn)[z[b].node0 + i + (size_t)(z[b].ni + 1) * j]; }
  double Y(int b, int i, int j) const { return (*in.yn)[z[b].node0 + i + (size_t)(z[b].ni + 1) * j]; }
  int cell(int b, int i, int j) const { return z[b].cell0 + i + z[b].ni * j; }
};

bool in_quad(const double* qx, const double* qy, double px, double py) {
  bool pos = false, neg = false;
  for (int k = 0; k < 4; ++k) {
    const int k1 = (k + 1) % 4;
    const double cr = (qx[k1] - qx[k]) * (py - qy[k]) - (qy[k1] - qy[k]) * (px - qx[k]);
    pos = pos || (cr > 0.0);
    neg = neg || (cr < 0.0);
  }
  return !(pos && neg);
}

double seg_d2(double px, double py, double ax, double ay, double bx, double by) {
  const double ex = bx - ax, ey = by - ay;
  const double l2 = ex * ex + ey * ey;
  double t = 0.0;
  if (l2 > 0.0) {
    t = ((px - ax) * ex + (py - ay) * ey) / l2;
    t = (t < 0.0) ? 0.0 : t;
    t = (t > 1.0) ? 1.0 : t;
  }
  const double dx = px - (ax + t * ex), dy = py - (ay + t * ey);
  return dx * dx + dy * dy;
}

// nodes along wall side s of zone b
void side_nodes(const Ctx& C, int b, int s, std::vector<double>& x, std::vector<double>& y) {
  const Zone& Z = C.z[b];
  const int n = (s < 2) ? Z.nj + 1 : Z.ni + 1;
  x.resize(n);
  y.resize(n);
  for (int m = 0; m < n; ++m) {
    const int i = (s == 0) ? 0 : (s == 1) ? Z.ni : m;
    const int j = (s == 2) ? 0 : (s == 3) ? Z.nj : m;
    x[m] = C.X(b, i, j);
    y[m] = C.Y(b, i, j);
  }
}

struct Walls {
  // per zone: polylines of its wall sides; closed outlines flagged
  std::vector<std::vector<std::vector<double>>> xs, ys;
  std::vector<std::vector<char>> closed;
  std::vector<std::vector<double>> ylo, yhi;  // y range of each polyline
};

Walls collect_walls(const Ctx& C) {
  Walls W;
  const int nb = (int)C.z.size();
  W.xs.resize(nb); W.ys.resize(nb); W.closed.resize(nb); W.ylo.resize(nb); W.yhi.resize(nb);
  for (int b = 0; b < nb; ++b) {
    const Zone& Z = C.z[b];
    for (int s = 0; s < 4; ++s) {
      if (Z.bc[s] != UGKS_BC_WALL) continue;
      std::vector<double> x, y;
      side_nodes(C, b, s, x, y);
      const bool cl = (s < 2) ? Z.bc[2] == UGKS_BC_PERIODIC : Z.bc[0] == UGKS_BC_PERIODIC;
      W.ylo[b].push_back(*std::min_element(y.begin(), y.end()));
      W.yhi[b].push_back(*std::max_element(y.begin(), y.end()));
      W.xs[b].push_back(std::move(x));
      W.ys[b].push_back(std::move(y));
      W.closed[b].push_back(cl ? 1 : 0);
    }
  }
  return W;
}

double wall_d2(const Walls& W, int b, double px, double py) {
  double d2 = std::numeric_limits<double>::infinity();
  for (size_t p = 0; p < W.xs[b].size(); ++p) {
    const auto& x = W.xs[b][p];
    const auto& y = W.ys[b][p];
    for (size_t m = 0; m + 1 < x.size(); ++m) d2 = std::min(d2, seg_d2(px, py, x[m], y[m], x[m + 1], y[m + 1]));
  }
  return d2;
}

bool in_body(const Walls& W, int self, double px, double py) {
  for (size_t b = 0; b < W.xs.size(); ++b) {
    if ((int)b == self) continue;
    for (size_t p = 0; p < W.xs[b].size(); ++p) {
      if (!W.closed[b][p]) continue;
      // no edge toggles outside the outline's y range
      if (py < W.ylo[b][p] || py >= W.yhi[b][p]) continue;
      const auto& x = W.xs[b][p];
      const auto& y = W.ys[b][p];
      bool in = false;
      for (size_t m = 0; m + 1 < x.size(); ++m) {
        const double ax = x[m], ay = y[m], ex = x[m + 1], ey = y[m + 1];
        if ((ay > py) != (ey > py)) {
          const double xi = ax + (py - ay) * (ex - ax) / (ey - ay);
          if (px < xi) in = !in;
        }
      }
      if (in) return true;
    }
  }
  return false;
}

void quad_of(const Ctx& C, int b, int n, double* qx, double* qy) {
  const Zone& Z = C.z[b];
  const int r = n - Z.cell0, i = r % Z.ni, j = r / Z.ni;
  qx[0] = C.X(b, i, j);         qy[0] = C.Y(b, i, j);
  qx[1] = C.X(b, i + 1, j);     qy[1] = C.Y(b, i + 1, j);
  qx[2] = C.X(b, i + 1, j + 1); qy[2] = C.Y(b, i + 1, j + 1);
  qx[3] = C.X(b, i, j + 1);     qy[3] = C.Y(b, i, j + 1);
}

int bucket_x(const Zone& Z, double x) {
  const int k = (int)std::floor((x - Z.x0) / Z.dx);
  return std::min(std::max(k, 0), Z.nbx - 1);
}
int bucket_y(const Zone& Z, double y) {
  const int k = (int)std::floor((y - Z.y0) / Z.dy);
  return std::min(std::max(k, 0), Z.nby - 1);
}

void build_buckets(Ctx& C, int b) {
  Zone& Z = C.z[b];
  Z.x0 = Z.y0 = std::numeric_limits<double>::infinity();
  Z.x1 = Z.y1 = -std::numeric_limits<double>::infinity();
  for (int j = 0; j <= Z.nj; ++j)
    for (int i = 0; i <= Z.ni; ++i) {
      Z.x0 = std::min(Z.x0, C.X(b, i, j)); Z.x1 = std::max(Z.x1, C.X(b, i, j));
      Z.y0 = std::min(Z.y0, C.Y(b, i, j)); Z.y1 = std::max(Z.y1, C.Y(b, i, j));
    }
  // margin: the pruning must keep every cell the rounded point-in-quad test
  // could accept, so boxes are widened by far more than a rounding error
  Z.eps = 1e-9 * std::max(Z.x1 - Z.x0, Z.y1 - Z.y0) + 1e-300;
  Z.x0 -= Z.eps; Z.y0 -= Z.eps; Z.x1 += Z.eps; Z.y1 += Z.eps;
  const int ncell = Z.ni * Z.nj;
  const int nside = std::max(1, (int)std::sqrt((double)ncell / 4.0));
  Z.nbx = Z.nby = nside;
  Z.dx = (Z.x1 > Z.x0) ? (Z.x1 - Z.x0) / nside : 1.0;
  Z.dy = (Z.y1 > Z.y0) ? (Z.y1 - Z.y0) / nside : 1.0;
  std::vector<int> cnt(Z.nbx * Z.nby + 1, 0);
  std::vector<int> rng(4 * (size_t)ncell);
  for (int r = 0; r < ncell; ++r) {
    double qx[4], qy[4];
    quad_of(C, b, Z.cell0 + r, qx, qy);
    const double xa = std::min(std::min(qx[0], qx[1]), std::min(qx[2], qx[3]));
    const double xb = std::max(std::max(qx[0], qx[1]), std::max(qx[2], qx[3]));
    const double ya = std::min(std::min(qy[0], qy[1]), std::min(qy[2], qy[3]));
    const double yb = std::max(std::max(qy[0], qy[1]), std::max(qy[2], qy[3]));
    int* R = &rng[4 * (size_t)r];
    R[0] = bucket_x(Z, xa - Z.eps); R[1] = bucket_x(Z, xb + Z.eps);
    R[2] = bucket_y(Z, ya - Z.eps); R[3] = bucket_y(Z, yb + Z.eps);
    for (int by = R[2]; by <= R[3]; ++by)
      for (int bx = R[0]; bx <= R[1]; ++bx) ++cnt[bx + Z.nbx * by + 1];
  }
  for (size_t k = 1; k < cnt.size(); ++k) cnt[k] += cnt[k - 1];
  Z.start = cnt;
  Z.items.assign(cnt.back(), 0);
  std::vector<int> fill(cnt.begin(), cnt.end() - 1);
  for (int r = 0; r < ncell; ++r) {  // ascending cell order within each bucket
    const int* R = &rng[4 * (size_t)r];
    for (int by = R[2]; by <= R[3]; ++by)
      for (int bx = R[0]; bx <= R[1]; ++bx) Z.items[fill[bx + Z.nbx * by]++] = Z.cell0 + r;
  }
}

// lowest cell of zone b containing p (field cells only when `ty` is given)
int locate(const Ctx& C, int b, double px, double py, const std::vector<signed char>* ty) {
  const Zone& Z = C.z[b];
  if (!(px >= Z.x0 && px <= Z.x1 && py >= Z.y0 && py <= Z.y1)) return -1;
  const int k = bucket_x(Z, px) + Z.nbx * bucket_y(Z, py);
  for (int e = Z.start[k]; e < Z.start[k + 1]; ++e) {
    const int n = Z.items[e];
    if (ty && (*ty)[n] != UGKS_FIELD) continue;
    double qx[4], qy[4];
    quad_of(C, b, n, qx, qy);
    if (in_quad(qx, qy, px, py)) return n;
  }
  return -1;
}

int depth(const Ctx& C, int b, int n) {
  const Zone& Z = C.z[b];
  const int r = n - Z.cell0, i = r % Z.ni, j = r / Z.ni;
  int d = kBig;
  if (Z.bc[0] == UGKS_BC_NONE) d = std::min(d, i);
  if (Z.bc[1] == UGKS_BC_NONE) d = std::min(d, Z.ni - 1 - i);
  if (Z.bc[2] == UGKS_BC_NONE) d = std::min(d, j);
  if (Z.bc[3] == UGKS_BC_NONE) d = std::min(d, Z.nj - 1 - j);
  return d;
}

// index neighbour inside the zone (periodic wrap) or -1
int nb_index(const Ctx& C, int b, int n, int dir, int side) {
  const Zone& Z = C.z[b];
  const int r = n - Z.cell0;
  int i = r % Z.ni, j = r / Z.ni;
  if (dir == 0) {
    i += side;
    if (i < 0 || i >= Z.ni) {
      if (Z.bc[0] != UGKS_BC_PERIODIC) return -1;
      i = (i + Z.ni) % Z.ni;
    }
  } else {
    j += side;
    if (j < 0 || j >= Z.nj) {
      if (Z.bc[2] != UGKS_BC_PERIODIC) return -1;
      j = (j + Z.nj) % Z.nj;
    }
  }
  return C.cell(b, i, j);
}

// donors and weights of cell n appended to `out`; false if it has no donor
bool donor_row(const Ctx& C, const std::vector<int>& zone_of, const std::vector<signed char>& ty,
               const std::vector<double>& cx, const std::vector<double>& cy, const std::vector<double>& vol,
               int n, int wrule, OversetOutput& out) {
  const int nb = (int)C.z.size();
  const double px = cx[n], py = cy[n];
  int d = -1, dz = -1;
  for (int z = 0; z < nb && d < 0; ++z)
    if (z != zone_of[n]) { d = locate(C, z, px, py, &ty); dz = z; }
  if (d < 0) return false;
  if (wrule == 1) {
    for (int q = 0; q < 4; ++q) {
      const int a = q % 2, bb = q / 2;
      const int lo_i = (a == 0) ? nb_index(C, dz, d, 0, -1) : d;
      const int c00 = (lo_i < 0) ? -1 : ((bb == 0) ? nb_index(C, dz, lo_i, 1, -1) : lo_i);
      if (c00 < 0) continue;
      const int c10 = nb_index(C, dz, c00, 0, +1);
      const int c01 = nb_index(C, dz, c00, 1, +1);
      const int c11 = (c10 < 0) ? -1 : nb_index(C, dz, c10, 1, +1);
      const int nq[4] = {c00, c10, c11, c01};
      bool ok = true;
      for (int k = 0; k < 4; ++k) ok = ok && nq[k] >= 0 && ty[nq[k]] == UGKS_FIELD;
      if (!ok) continue;
      double qx[4], qy[4];
      for (int k = 0; k < 4; ++k) { qx[k] = cx[nq[k]]; qy[k] = cy[nq[k]]; }
      if (!in_quad(qx, qy, px, py)) continue;
      // inverse bilinear map: three Newton steps from the middle of the quad
      double s = 0.5, t = 0.5;
      for (int it = 0; it < 3; ++it) {
        const double rx = (1.0 - s) * (1.0 - t) * qx[0] + s * (1.0 - t) * qx[1] + s * t * qx[2] +
                          (1.0 - s) * t * qx[3] - px;
        const double ry = (1.0 - s) * (1.0 - t) * qy[0] + s * (1.0 - t) * qy[1] + s * t * qy[2] +
                          (1.0 - s) * t * qy[3] - py;
        const double xs = (1.0 - t) * (qx[1] - qx[0]) + t * (qx[2] - qx[3]);
        const double ys = (1.0 - t) * (qy[1] - qy[0]) + t * (qy[2] - qy[3]);
        const double xt = (1.0 - s) * (qx[3] - qx[0]) + s * (qx[2] - qx[1]);
        const double yt = (1.0 - s) * (qy[3] - qy[0]) + s * (qy[2] - qy[1]);
        const double det = xs * yt - xt * ys;
        s -= (rx * yt - xt * ry) / det;
        t -= (xs * ry - rx * ys) / det;
      }
      const double wq[4] = {(1.0 - s) * (1.0 - t), s * (1.0 - t), s * t, (1.0 - s) * t};
      for (int k = 0; k < 4; ++k) { out.don.push_back(nq[k]); out.w.push_back(wq[k]); }
      return true;
    }
  }
  int set[5], ns = 0;
  set[ns++] = d;
  for (int dir = 0; dir < 2; ++dir)
    for (int sd = -1; sd <= 1; sd += 2) {
      const int m = nb_index(C, dz, d, dir, sd);
      if (m < 0 || ty[m] != UGKS_FIELD) continue;
      if (std::find(set, set + ns, m) == set + ns) set[ns++] = m;
    }
  double d2[5];
  int exact = -1;
  for (int k = 0; k < ns; ++k) {
    const double ex = cx[set[k]] - px, ey = cy[set[k]] - py;
    d2[k] = ex * ex + ey * ey;
    if (exact < 0 && d2[k] <= 1e-28 * vol[set[k]]) exact = k;
  }
  if (exact >= 0) {
    out.don.push_back(set[exact]);
    out.w.push_back(1.0);
    return true;
  }
  double sum = 0.0;
  for (int k = 0; k < ns; ++k) sum += 1.0 / d2[k];
  for (int k = 0; k < ns; ++k) { out.don.push_back(set[k]); out.w.push_back((1.0 / d2[k]) / sum); }
  return true;
}

}  // namespace

int overset_build(const OversetInput& in, int wrule, int overlap, OversetOutput& out, std::string& msg) {
  Ctx C(in);
  const int nb = in.nblock;
  int ncell = 0;
  C.z.resize(nb);
  std::vector<int> zone_of;
  for (int b = 0; b < nb; ++b) {
    Zone& Z = C.z[b];
    Z.ni = in.ni[b]; Z.nj = in.nj[b]; Z.cell0 = in.cell0[b]; Z.node0 = (*in.node0)[b];
    for (int s = 0; s < 4; ++s) Z.bc[s] = in.bc[4 * b + s];
    ncell += Z.ni * Z.nj;
  }
  zone_of.resize(ncell);
  for (int b = 0; b < nb; ++b)
    for (int r = 0; r < C.z[b].ni * C.z[b].nj; ++r) zone_of[C.z[b].cell0 + r] = b;
  for (int b = 0; b < nb; ++b) build_buckets(C, b);
  const Walls W = collect_walls(C);
  const int cut = overlap + 3;
  // node classes
  // (every node on its own: node rows of a zone are shared among threads)
  std::vector<std::vector<char>> off(nb);
  const int nthr = (int)std::min(16u, std::max(1u, std::thread::hardware_concurrency()));
  for (int b = 0; b < nb; ++b) {
    const Zone& Z = C.z[b];
    off[b].assign((size_t)(Z.ni + 1) * (Z.nj + 1), 0);
    auto rows = [&](int j0) {
      for (int j = j0; j <= Z.nj; j += nthr)
        for (int i = 0; i <= Z.ni; ++i) {
          const double px = C.X(b, i, j), py = C.Y(b, i, j);
          bool o = in_body(W, b, px, py);
          // the own wall distance only where another zone covers the node
          double da = -1.0;
          for (int z = 0; z < nb && !o; ++z) {
            if (z == b) continue;
            const int m = locate(C, z, px, py, nullptr);
            if (m < 0 || depth(C, z, m) < cut) continue;
            if (da < 0.0) da = wall_d2(W, b, px, py);
            const double dz = wall_d2(W, z, px, py);
            o = (dz < da) || (dz == da && z > b);
          }
          off[b][i + (size_t)(Z.ni + 1) * j] = o ? 1 : 0;
        }
    };
    std::vector<std::thread> pool;
    for (int t = 1; t < nthr; ++t) pool.emplace_back(rows, t);
    rows(0);
    for (auto& th : pool) th.join();
  }
  // cell classes
  std::vector<signed char> cls(ncell);
  for (int b = 0; b < nb; ++b) {
    const Zone& Z = C.z[b];
    const auto& O = off[b];
    for (int j = 0; j < Z.nj; ++j)
      for (int i = 0; i < Z.ni; ++i) {
        const size_t w = Z.ni + 1;
        const int k = O[i + w * j] + O[i + 1 + w * j] + O[i + 1 + w * (j + 1)] + O[i + w * (j + 1)];
        cls[C.cell(b, i, j)] = (k == 0) ? UGKS_FIELD : (k == 4) ? UGKS_HOLE : UGKS_RECEPTOR;
      }
  }
  // receptors: boundary, buffer layer, fringe beside overset sides
  std::vector<signed char>& ty = out.type;
  ty = cls;
  for (int n = 0; n < ncell; ++n) {
    if (cls[n] != UGKS_FIELD) continue;
    const int b = zone_of[n];
    const Zone& Z = C.z[b];
    for (int dir = 0; dir < 2; ++dir)
      for (int sd = -1; sd <= 1; sd += 2) {
        const int m = nb_index(C, b, n, dir, sd);
        if (m >= 0 && cls[m] != UGKS_FIELD) ty[n] = UGKS_RECEPTOR;
      }
    const int r = n - Z.cell0, i = r % Z.ni, j = r / Z.ni;
    if ((Z.bc[0] == UGKS_BC_NONE && i < overlap) || (Z.bc[1] == UGKS_BC_NONE && i >= Z.ni - overlap) ||
        (Z.bc[2] == UGKS_BC_NONE && j < overlap) || (Z.bc[3] == UGKS_BC_NONE && j >= Z.nj - overlap))
      ty[n] = UGKS_RECEPTOR;
  }
  // donors and weights: receptors, then the cells uncovered from holes
  const auto& cx = *in.cx;
  const auto& cy = *in.cy;
  const auto& vol = *in.vol;
  out.rec.clear(); out.don.clear(); out.w.clear();
  out.ptr.assign(1, 0);
  out.nrec = 0;
  // cells uncovered from holes take donors among the cells that were not
  // holes, so that they can be filled before the receptors (which may use
  // them as donors)
  auto uncovered = [&](int n) { return in.old_type && (*in.old_type)[n] == UGKS_HOLE && ty[n] == UGKS_FIELD; };
  std::vector<signed char> tyr(ty);
  for (int n = 0; n < ncell; ++n)
    if (uncovered(n)) tyr[n] = UGKS_HOLE;
  for (int pass = 0; pass < 2; ++pass)
    for (int n = 0; n < ncell; ++n) {
      const bool want = (pass == 0) ? ty[n] == UGKS_RECEPTOR : uncovered(n);
      if (!want) continue;
      if (!donor_row(C, zone_of, (pass == 0) ? ty : tyr, cx, cy, vol, n, wrule, out)) {
        msg = "overset cell " + std::to_string(n) + " has no donor";
        return UGKS_E_ORPHAN;
      }
      out.rec.push_back(n);
      out.ptr.push_back((int)out.don.size());
      if (pass == 0) ++out.nrec;
    }
  return UGKS_OK;
}

}  // namespace ugks
