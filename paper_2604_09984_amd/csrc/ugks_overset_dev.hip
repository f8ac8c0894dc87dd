// Device overset assembly of libugks (Sec. 3.1 mesh assembly, Sec. 3.2
// interpolation weights): the same rules and predicates as the host
// assembly (ugks_overset.cpp), evaluated on the GPU with the same
// floating-point expressions and no contraction (this file is compiled with
// -ffp-contract=off), so that node classes, cell kinds, receptors, donors and
// weights are identical bit for bit.
//
//   1. bins: each zone's bounding box cut into a uniform grid of bins; every
//      cell is listed in the bins its widened box overlaps (counted, scanned
//      and filled with atomics: the order inside a bin is arbitrary, so a
//      point search takes the lowest containing cell of all candidates,
//      which is the first one of an ordered scan);
//   2. node classes, one thread per node: inside another zone's closed wall
//      outline (crossing number), or covered by another zone's cell lying at
//      least overlap + 3 layers inside its overset sides and nearer to that
//      zone's walls (ties: the higher zone);
//   3. cell kinds from the four node classes, receptors (boundary cells, one
//      buffer layer, `overlap` layers beside overset sides);
//   4. donors, one thread per receptor (and per cell uncovered from a hole):
//      the lowest-zone, lowest-index field cell containing the centroid;
//      inverse-distance or bilinear weights;
//   5. rows compacted by exclusive scans in the host order (receptors by
//      cell, then the uncovered cells by cell).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <limits>
#include <string>

#include "ugks.h"
#include "ugks_overset.h"

namespace ugks {
namespace {

constexpr int kBigDepth = 1 << 30;
constexpr int kMaxDon = 5;
const int kNoOrphan = 0x7fffffff;

// zone table on the device
struct DZone {
  int ni, nj, cell0, bc[4];
  long long node0;
  double x0, y0, x1, y1, dx, dy, eps;
  int nbx, nby, bin0;  // bins of this zone start at bin0 in the global bin arrays
  int poly0, npoly;    // wall polylines of this zone
};
struct DPoly {
  int off, len, closed;
  double ylo, yhi;
};
struct DGeo {
  int nzone, ncell;
  const DZone* z;
  const DPoly* poly;
  const double *wx, *wy;  // wall polyline nodes
  const double *xn, *yn;  // nodes, zones concatenated
  const double *cx, *cy, *vol;
  const int *bstart, *bitem;
};

__device__ __forceinline__ double gx(const DGeo& G, const DZone& Z, int i, int j) {
  return G.xn[Z.node0 + i + (long long)(Z.ni + 1) * j];
}
__device__ __forceinline__ double gy(const DGeo& G, const DZone& Z, int i, int j) {
  return G.yn[Z.node0 + i + (long long)(Z.ni + 1) * j];
}

__device__ bool d_in_quad(const double* qx, const double* qy, double px, double py) {
#pragma clang fp contract(off)
  bool pos = false, neg = false;
  for (int k = 0; k < 4; ++k) {
    const int k1 = (k + 1) % 4;
    const double cr = (qx[k1] - qx[k]) * (py - qy[k]) - (qy[k1] - qy[k]) * (px - qx[k]);
    pos = pos || (cr > 0.0);
    neg = neg || (cr < 0.0);
  }
  return !(pos && neg);
}

__device__ double d_seg_d2(double px, double py, double ax, double ay, double bx, double by) {
#pragma clang fp contract(off)
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

__device__ double d_wall_d2(const DGeo& G, int b, double px, double py) {
  double d2 = __builtin_inf();
  const DZone& Z = G.z[b];
  for (int p = Z.poly0; p < Z.poly0 + Z.npoly; ++p) {
    const DPoly& P = G.poly[p];
    for (int m = 0; m + 1 < P.len; ++m) {
      const double s = d_seg_d2(px, py, G.wx[P.off + m], G.wy[P.off + m], G.wx[P.off + m + 1], G.wy[P.off + m + 1]);
      d2 = (s < d2) ? s : d2;
    }
  }
  return d2;
}

__device__ bool d_in_body(const DGeo& G, int self, double px, double py) {
#pragma clang fp contract(off)
  for (int b = 0; b < G.nzone; ++b) {
    if (b == self) continue;
    const DZone& Z = G.z[b];
    for (int p = Z.poly0; p < Z.poly0 + Z.npoly; ++p) {
      const DPoly& P = G.poly[p];
      if (!P.closed) continue;
      if (py < P.ylo || py >= P.yhi) continue;
      bool in = false;
      for (int m = 0; m + 1 < P.len; ++m) {
        const double ax = G.wx[P.off + m], ay = G.wy[P.off + m], ex = G.wx[P.off + m + 1], ey = G.wy[P.off + m + 1];
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

__device__ void d_quad_of(const DGeo& G, const DZone& Z, int n, double* qx, double* qy) {
  const int r = n - Z.cell0, i = r % Z.ni, j = r / Z.ni;
  qx[0] = gx(G, Z, i, j);         qy[0] = gy(G, Z, i, j);
  qx[1] = gx(G, Z, i + 1, j);     qy[1] = gy(G, Z, i + 1, j);
  qx[2] = gx(G, Z, i + 1, j + 1); qy[2] = gy(G, Z, i + 1, j + 1);
  qx[3] = gx(G, Z, i, j + 1);     qy[3] = gy(G, Z, i, j + 1);
}

__device__ __forceinline__ int d_bin_x(const DZone& Z, double x) {
  const int k = (int)floor((x - Z.x0) / Z.dx);
  return min(max(k, 0), Z.nbx - 1);
}
__device__ __forceinline__ int d_bin_y(const DZone& Z, double y) {
  const int k = (int)floor((y - Z.y0) / Z.dy);
  return min(max(k, 0), Z.nby - 1);
}

// lowest cell of zone b containing p (field cells only when ty is given)
__device__ int d_locate(const DGeo& G, int b, double px, double py, const signed char* ty) {
  const DZone& Z = G.z[b];
  if (!(px >= Z.x0 && px <= Z.x1 && py >= Z.y0 && py <= Z.y1)) return -1;
  const int k = Z.bin0 + d_bin_x(Z, px) + Z.nbx * d_bin_y(Z, py);
  int best = -1;
  for (int e = G.bstart[k]; e < G.bstart[k + 1]; ++e) {
    const int n = G.bitem[e];
    if (best >= 0 && n >= best) continue;
    if (ty && ty[n] != UGKS_FIELD) continue;
    double qx[4], qy[4];
    d_quad_of(G, Z, n, qx, qy);
    if (d_in_quad(qx, qy, px, py)) best = n;
  }
  return best;
}

__device__ int d_depth(const DZone& Z, int n) {
  const int r = n - Z.cell0, i = r % Z.ni, j = r / Z.ni;
  int d = kBigDepth;
  if (Z.bc[0] == UGKS_BC_NONE) d = min(d, i);
  if (Z.bc[1] == UGKS_BC_NONE) d = min(d, Z.ni - 1 - i);
  if (Z.bc[2] == UGKS_BC_NONE) d = min(d, j);
  if (Z.bc[3] == UGKS_BC_NONE) d = min(d, Z.nj - 1 - j);
  return d;
}

__device__ int d_nb_index(const DZone& Z, int n, int dir, int side) {
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
  return Z.cell0 + i + Z.ni * j;
}

__device__ int zone_of_cell(const DGeo& G, int n) {
  int b = 0;
  while (b + 1 < G.nzone && G.z[b + 1].cell0 <= n) ++b;
  return b;
}

// 1. bins: per cell, the range of bins its widened box overlaps; counted
__global__ void k_bin_count(DGeo G, int* __restrict__ cnt, int4* __restrict__ rng) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= G.ncell) return;
  const DZone& Z = G.z[zone_of_cell(G, n)];
  double qx[4], qy[4];
  d_quad_of(G, Z, n, qx, qy);
  const double xa = fmin(fmin(qx[0], qx[1]), fmin(qx[2], qx[3]));
  const double xb = fmax(fmax(qx[0], qx[1]), fmax(qx[2], qx[3]));
  const double ya = fmin(fmin(qy[0], qy[1]), fmin(qy[2], qy[3]));
  const double yb = fmax(fmax(qy[0], qy[1]), fmax(qy[2], qy[3]));
  const int4 R = make_int4(d_bin_x(Z, xa - Z.eps), d_bin_x(Z, xb + Z.eps), d_bin_y(Z, ya - Z.eps), d_bin_y(Z, yb + Z.eps));
  rng[n] = R;
  for (int by = R.z; by <= R.w; ++by)
    for (int bx = R.x; bx <= R.y; ++bx) atomicAdd(&cnt[Z.bin0 + bx + Z.nbx * by], 1);
}
__global__ void k_bin_fill(DGeo G, const int4* __restrict__ rng, int* __restrict__ fill, int* __restrict__ item) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= G.ncell) return;
  const DZone& Z = G.z[zone_of_cell(G, n)];
  const int4 R = rng[n];
  for (int by = R.z; by <= R.w; ++by)
    for (int bx = R.x; bx <= R.y; ++bx) item[atomicAdd(&fill[Z.bin0 + bx + Z.nbx * by], 1)] = n;
}

// 2. node classes (1: inactive)
__global__ void k_node_class(DGeo G, long long nnode, int cut, signed char* __restrict__ off) {
#pragma clang fp contract(off)
  const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nnode) return;
  int b = 0;
  while (b + 1 < G.nzone && G.z[b + 1].node0 <= v) ++b;
  const DZone& Z = G.z[b];
  const long long r = v - Z.node0;
  const int i = (int)(r % (Z.ni + 1)), j = (int)(r / (Z.ni + 1));
  const double px = gx(G, Z, i, j), py = gy(G, Z, i, j);
  bool o = d_in_body(G, b, px, py);
  double da = -1.0;
  for (int z = 0; z < G.nzone && !o; ++z) {
    if (z == b) continue;
    const int m = d_locate(G, z, px, py, nullptr);
    if (m < 0 || d_depth(G.z[z], m) < cut) continue;
    if (da < 0.0) da = d_wall_d2(G, b, px, py);
    const double dz = d_wall_d2(G, z, px, py);
    o = (dz < da) || (dz == da && z > b);
  }
  off[v] = o ? 1 : 0;
}

// 3. cell classes, then kinds with the receptor layers; want: 1 receptor
// row, 2 uncovered cell (was a hole, is field now)
__global__ void k_cell_class(DGeo G, const signed char* __restrict__ off, signed char* __restrict__ cls) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= G.ncell) return;
  const DZone& Z = G.z[zone_of_cell(G, n)];
  const int r = n - Z.cell0, i = r % Z.ni, j = r / Z.ni;
  const long long w = Z.ni + 1;
  const signed char* O = off + Z.node0;
  const int k = O[i + w * j] + O[i + 1 + w * j] + O[i + 1 + w * (j + 1)] + O[i + w * (j + 1)];
  cls[n] = (k == 0) ? UGKS_FIELD : (k == 4) ? UGKS_HOLE : UGKS_RECEPTOR;
}
__global__ void k_cell_kind(DGeo G, int overlap, const signed char* __restrict__ cls,
                            const signed char* __restrict__ old_type, signed char* __restrict__ ty,
                            signed char* __restrict__ tyr, int* __restrict__ want0, int* __restrict__ want1) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= G.ncell) return;
  const DZone& Z = G.z[zone_of_cell(G, n)];
  signed char t = cls[n];
  if (t == UGKS_FIELD) {
    for (int dir = 0; dir < 2; ++dir)
      for (int sd = -1; sd <= 1; sd += 2) {
        const int m = d_nb_index(Z, n, dir, sd);
        if (m >= 0 && cls[m] != UGKS_FIELD) t = UGKS_RECEPTOR;
      }
    const int r = n - Z.cell0, i = r % Z.ni, j = r / Z.ni;
    if ((Z.bc[0] == UGKS_BC_NONE && i < overlap) || (Z.bc[1] == UGKS_BC_NONE && i >= Z.ni - overlap) ||
        (Z.bc[2] == UGKS_BC_NONE && j < overlap) || (Z.bc[3] == UGKS_BC_NONE && j >= Z.nj - overlap))
      t = UGKS_RECEPTOR;
  }
  ty[n] = t;
  const bool unc = old_type[n] == UGKS_HOLE && t == UGKS_FIELD;
  tyr[n] = unc ? (signed char)UGKS_HOLE : t;
  want0[n] = (t == UGKS_RECEPTOR) ? 1 : 0;
  want1[n] = unc ? 1 : 0;
}

// 4. donors and weights of the wanted cells (the rule of the host's
// donor_row); cnt[n] = number of donors, 0 if not wanted; *orphan becomes
// the lowest wanted cell without donor
__global__ void k_donors(DGeo G, int wrule, const signed char* __restrict__ ty, const signed char* __restrict__ tyr,
                         const int* __restrict__ want0, const int* __restrict__ want1, int* __restrict__ cnt,
                         int* __restrict__ don, double* __restrict__ wgt, int* __restrict__ orphan) {
#pragma clang fp contract(off)
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= G.ncell) return;
  cnt[n] = 0;
  if (!want0[n] && !want1[n]) return;
  const signed char* T = want0[n] ? ty : tyr;
  const int self = zone_of_cell(G, n);
  const double px = G.cx[n], py = G.cy[n];
  int d = -1, dz = -1;
  for (int z = 0; z < G.nzone && d < 0; ++z)
    if (z != self) { d = d_locate(G, z, px, py, T); dz = z; }
  if (d < 0) { atomicMin(orphan, n); return; }
  const DZone& Z = G.z[dz];
  int* od = don + (size_t)kMaxDon * n;
  double* ow = wgt + (size_t)kMaxDon * n;
  if (wrule == 1) {
    for (int q = 0; q < 4; ++q) {
      const int a = q % 2, bb = q / 2;
      const int lo_i = (a == 0) ? d_nb_index(Z, d, 0, -1) : d;
      const int c00 = (lo_i < 0) ? -1 : ((bb == 0) ? d_nb_index(Z, lo_i, 1, -1) : lo_i);
      if (c00 < 0) continue;
      const int c10 = d_nb_index(Z, c00, 0, +1);
      const int c01 = d_nb_index(Z, c00, 1, +1);
      const int c11 = (c10 < 0) ? -1 : d_nb_index(Z, c10, 1, +1);
      const int nq[4] = {c00, c10, c11, c01};
      bool ok = true;
      for (int k = 0; k < 4; ++k) ok = ok && nq[k] >= 0 && T[nq[k]] == UGKS_FIELD;
      if (!ok) continue;
      double qx[4], qy[4];
      for (int k = 0; k < 4; ++k) { qx[k] = G.cx[nq[k]]; qy[k] = G.cy[nq[k]]; }
      if (!d_in_quad(qx, qy, px, py)) continue;
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
      for (int k = 0; k < 4; ++k) { od[k] = nq[k]; ow[k] = wq[k]; }
      cnt[n] = 4;
      return;
    }
  }
  int set[kMaxDon], ns = 0;
  set[ns++] = d;
  for (int dir = 0; dir < 2; ++dir)
    for (int sd = -1; sd <= 1; sd += 2) {
      const int m = d_nb_index(Z, d, dir, sd);
      if (m < 0 || T[m] != UGKS_FIELD) continue;
      bool seen = false;
      for (int k = 0; k < ns; ++k) seen = seen || set[k] == m;
      if (!seen) set[ns++] = m;
    }
  double d2[kMaxDon];
  int exact = -1;
  for (int k = 0; k < ns; ++k) {
    const double ex = G.cx[set[k]] - px, ey = G.cy[set[k]] - py;
    d2[k] = ex * ex + ey * ey;
    if (exact < 0 && d2[k] <= 1e-28 * G.vol[set[k]]) exact = k;
  }
  if (exact >= 0) {
    od[0] = set[exact];
    ow[0] = 1.0;
    cnt[n] = 1;
    return;
  }
  double sum = 0.0;
  for (int k = 0; k < ns; ++k) sum += 1.0 / d2[k];
  for (int k = 0; k < ns; ++k) { od[k] = set[k]; ow[k] = (1.0 / d2[k]) / sum; }
  cnt[n] = ns;
}

// exclusive scan of n ints in place (chunks of 1024 scanned per workgroup,
// then the chunk sums by one workgroup, then added back); out[n] = total
constexpr int kScanB = 1024;
__global__ void k_scan_chunks(const int* __restrict__ in, int* __restrict__ out, int* __restrict__ sums, int n,
                              const int* __restrict__ mask) {
  __shared__ int s[kScanB];
  const int t = threadIdx.x, i = blockIdx.x * kScanB + t;
  int v = (i < n) ? in[i] : 0;
  if (mask && i < n && !mask[i]) v = 0;
  s[t] = v;
  __syncthreads();
  for (int o = 1; o < kScanB; o <<= 1) {
    const int a = (t >= o) ? s[t - o] : 0;
    __syncthreads();
    s[t] += a;
    __syncthreads();
  }
  if (i < n) out[i] = s[t] - v;
  if (t == kScanB - 1) sums[blockIdx.x] = s[t];
}
__global__ void k_scan_sums(int* __restrict__ sums, int nchunk, int base, int* __restrict__ total) {
  if (threadIdx.x != 0) return;
  int acc = base;
  for (int k = 0; k < nchunk; ++k) {
    const int v = sums[k];
    sums[k] = acc;
    acc += v;
  }
  *total = acc;
}
__global__ void k_scan_add(int* __restrict__ out, const int* __restrict__ sums, int n) {
  const int i = blockIdx.x * kScanB + threadIdx.x;
  if (i < n) out[i] += sums[blockIdx.x];
}

// 5. rows: rec[row] = n, ptr[row + 1] = end of its donors, donors and weights
__global__ void k_rows(int ncell, const int* __restrict__ want0, const int* __restrict__ want1,
                       const int* __restrict__ row0, const int* __restrict__ row1, const int* __restrict__ doff0,
                       const int* __restrict__ doff1, const int* __restrict__ cnt, const int* __restrict__ don,
                       const double* __restrict__ wgt, int* __restrict__ rec, int* __restrict__ ptr,
                       int* __restrict__ odon, double* __restrict__ ow) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= ncell || !(want0[n] || want1[n])) return;
  const int r = want0[n] ? row0[n] : row1[n];
  const int o = want0[n] ? doff0[n] : doff1[n];
  rec[r] = n;
  ptr[r + 1] = o + cnt[n];
  for (int k = 0; k < cnt[n]; ++k) {
    odon[o + k] = don[(size_t)kMaxDon * n + k];
    ow[o + k] = wgt[(size_t)kMaxDon * n + k];
  }
}

// device scratch of one assembly, freed on return
struct Scratch {
  std::vector<void*> p;
  ~Scratch() {
    for (void* q : p) (void)hipFree(q);
  }
  template <class X>
  X* get(size_t n) {
    void* q = nullptr;
    if (hipMalloc(&q, sizeof(X) * std::max<size_t>(n, 1)) != hipSuccess) return nullptr;
    p.push_back(q);
    return (X*)q;
  }
};

unsigned nblk(long long n, int t) { return (unsigned)((n + t - 1) / t); }

// exclusive scan of in (masked) into out starting at base; returns the total
int scan(const int* in, const int* mask, int* out, int n, int base, int* sums, int* total, hipStream_t st) {
  const int nchunk = (n + kScanB - 1) / kScanB;
  if (nchunk > 0) k_scan_chunks<<<nchunk, kScanB, 0, st>>>(in, out, sums, n, mask);
  k_scan_sums<<<1, 64, 0, st>>>(sums, nchunk, base, total);
  if (nchunk > 0) k_scan_add<<<nchunk, kScanB, 0, st>>>(out, sums, n);
  int h = 0;
  if (hipMemcpyAsync(&h, total, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return -1;
  return h;
}

}  // namespace

int overset_build_device(const OversetInput& in, int wrule, int overlap, OversetOutput& out, std::string& msg) {
  const int nb = in.nblock;
  int ncell = 0;
  for (int b = 0; b < nb; ++b) ncell += in.ni[b] * in.nj[b];
  const auto& xn = *in.xn;
  const auto& yn = *in.yn;
  const long long nnode = (long long)xn.size();
  // zone table, bins (bounding boxes and bin counts on the host: O(nodes)),
  // wall polylines
  std::vector<DZone> Z(nb);
  std::vector<DPoly> P;
  std::vector<double> wx, wy;
  int nbin = 0;
  for (int b = 0; b < nb; ++b) {
    DZone& z = Z[b];
    z.ni = in.ni[b]; z.nj = in.nj[b]; z.cell0 = in.cell0[b]; z.node0 = (long long)(*in.node0)[b];
    for (int s = 0; s < 4; ++s) z.bc[s] = in.bc[4 * b + s];
    z.x0 = z.y0 = std::numeric_limits<double>::infinity();
    z.x1 = z.y1 = -std::numeric_limits<double>::infinity();
    const long long nn = (long long)(z.ni + 1) * (z.nj + 1);
    for (long long v = z.node0; v < z.node0 + nn; ++v) {
      z.x0 = std::min(z.x0, xn[v]); z.x1 = std::max(z.x1, xn[v]);
      z.y0 = std::min(z.y0, yn[v]); z.y1 = std::max(z.y1, yn[v]);
    }
    z.eps = 1e-9 * std::max(z.x1 - z.x0, z.y1 - z.y0) + 1e-300;
    z.x0 -= z.eps; z.y0 -= z.eps; z.x1 += z.eps; z.y1 += z.eps;
    const int nside = std::max(1, (int)std::sqrt((double)(z.ni * z.nj) / 4.0));
    z.nbx = z.nby = nside;
    z.dx = (z.x1 > z.x0) ? (z.x1 - z.x0) / nside : 1.0;
    z.dy = (z.y1 > z.y0) ? (z.y1 - z.y0) / nside : 1.0;
    z.bin0 = nbin;
    nbin += nside * nside;
    z.poly0 = (int)P.size();
    for (int s = 0; s < 4; ++s) {
      if (z.bc[s] != UGKS_BC_WALL) continue;
      const int n = (s < 2) ? z.nj + 1 : z.ni + 1;
      DPoly q;
      q.off = (int)wx.size();
      q.len = n;
      q.closed = (s < 2) ? z.bc[2] == UGKS_BC_PERIODIC : z.bc[0] == UGKS_BC_PERIODIC;
      q.ylo = std::numeric_limits<double>::infinity();
      q.yhi = -std::numeric_limits<double>::infinity();
      for (int m = 0; m < n; ++m) {
        const int i = (s == 0) ? 0 : (s == 1) ? z.ni : m;
        const int j = (s == 2) ? 0 : (s == 3) ? z.nj : m;
        const long long v = z.node0 + i + (long long)(z.ni + 1) * j;
        wx.push_back(xn[v]);
        wy.push_back(yn[v]);
        q.ylo = std::min(q.ylo, yn[v]);
        q.yhi = std::max(q.yhi, yn[v]);
      }
      P.push_back(q);
    }
    z.npoly = (int)P.size() - z.poly0;
  }
  hipStream_t st = nullptr;
  if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
    msg = "stream creation failed";
    return UGKS_E_DEVICE;
  }
  struct StreamGuard {
    hipStream_t s;
    ~StreamGuard() { (void)hipStreamDestroy(s); }
  } guard{st};
  Scratch S;
  DZone* dz = S.get<DZone>(nb);
  DPoly* dp = S.get<DPoly>(P.size());
  double *dwx = S.get<double>(wx.size()), *dwy = S.get<double>(wy.size());
  double *dxn = S.get<double>(nnode), *dyn = S.get<double>(nnode);
  double *dcx = S.get<double>(ncell), *dcy = S.get<double>(ncell), *dvol = S.get<double>(ncell);
  signed char* dold = S.get<signed char>(ncell);
  int* bcnt = S.get<int>(nbin + 1);
  int* bstart = S.get<int>(nbin + 1);
  int4* rng = S.get<int4>(ncell);
  signed char* off = S.get<signed char>(nnode);
  signed char *cls = S.get<signed char>(ncell), *ty = S.get<signed char>(ncell), *tyr = S.get<signed char>(ncell);
  int *want0 = S.get<int>(ncell), *want1 = S.get<int>(ncell), *cnt = S.get<int>(ncell);
  int* don = S.get<int>((size_t)kMaxDon * ncell);
  double* wgt = S.get<double>((size_t)kMaxDon * ncell);
  int *row0 = S.get<int>(ncell), *row1 = S.get<int>(ncell), *doff0 = S.get<int>(ncell), *doff1 = S.get<int>(ncell);
  int* sums = S.get<int>((ncell + kScanB - 1) / kScanB + 1);
  int* scal = S.get<int>(4);  // orphan flag, scan total
  for (void* q : S.p)
    if (!q) {
      msg = "device allocation failed";
      return UGKS_E_DEVICE;
    }
  std::vector<signed char> old(ncell, UGKS_FIELD);
  if (in.old_type) old = *in.old_type;
  bool ok = hipMemcpyAsync(dz, Z.data(), sizeof(DZone) * nb, hipMemcpyHostToDevice, st) == hipSuccess &&
            (P.empty() || hipMemcpyAsync(dp, P.data(), sizeof(DPoly) * P.size(), hipMemcpyHostToDevice, st) == hipSuccess) &&
            (wx.empty() || hipMemcpyAsync(dwx, wx.data(), sizeof(double) * wx.size(), hipMemcpyHostToDevice, st) == hipSuccess) &&
            (wy.empty() || hipMemcpyAsync(dwy, wy.data(), sizeof(double) * wy.size(), hipMemcpyHostToDevice, st) == hipSuccess) &&
            hipMemcpyAsync(dxn, xn.data(), sizeof(double) * nnode, hipMemcpyHostToDevice, st) == hipSuccess &&
            hipMemcpyAsync(dyn, yn.data(), sizeof(double) * nnode, hipMemcpyHostToDevice, st) == hipSuccess &&
            hipMemcpyAsync(dcx, in.cx->data(), sizeof(double) * ncell, hipMemcpyHostToDevice, st) == hipSuccess &&
            hipMemcpyAsync(dcy, in.cy->data(), sizeof(double) * ncell, hipMemcpyHostToDevice, st) == hipSuccess &&
            hipMemcpyAsync(dvol, in.vol->data(), sizeof(double) * ncell, hipMemcpyHostToDevice, st) == hipSuccess &&
            hipMemcpyAsync(dold, old.data(), ncell, hipMemcpyHostToDevice, st) == hipSuccess &&
            hipMemsetAsync(bcnt, 0, sizeof(int) * (nbin + 1), st) == hipSuccess &&
            hipMemsetAsync(scal, 0, sizeof(int) * 4, st) == hipSuccess &&
            hipMemcpyAsync(scal, &kNoOrphan, sizeof(int), hipMemcpyHostToDevice, st) == hipSuccess;
  if (!ok) {
    msg = "upload of the assembly inputs failed";
    return UGKS_E_DEVICE;
  }
  DGeo G{nb, ncell, dz, dp, dwx, dwy, dxn, dyn, dcx, dcy, dvol, bstart, nullptr};
  // 1. bins
  k_bin_count<<<nblk(ncell, 256), 256, 0, st>>>(G, bcnt, rng);
  if (scan(bcnt, nullptr, bstart, nbin, 0, sums, scal + 1, st) < 0) {
    msg = "bin scan failed";
    return UGKS_E_DEVICE;
  }
  int nitem = 0;
  if (hipMemcpyAsync(bstart + nbin, scal + 1, sizeof(int), hipMemcpyDeviceToDevice, st) != hipSuccess ||
      hipMemcpyAsync(&nitem, scal + 1, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess) {
    msg = "bin scan failed";
    return UGKS_E_DEVICE;
  }
  int* bitem = S.get<int>(nitem);
  int* bfill = S.get<int>(nbin + 1);
  if (!bitem || !bfill ||
      hipMemcpyAsync(bfill, bstart, sizeof(int) * (nbin + 1), hipMemcpyDeviceToDevice, st) != hipSuccess) {
    msg = "device allocation failed";
    return UGKS_E_DEVICE;
  }
  k_bin_fill<<<nblk(ncell, 256), 256, 0, st>>>(G, rng, bfill, bitem);
  G.bitem = bitem;
  // 2.-4.
  k_node_class<<<nblk(nnode, 128), 128, 0, st>>>(G, nnode, overlap + 3, off);
  k_cell_class<<<nblk(ncell, 256), 256, 0, st>>>(G, off, cls);
  k_cell_kind<<<nblk(ncell, 256), 256, 0, st>>>(G, overlap, cls, dold, ty, tyr, want0, want1);
  k_donors<<<nblk(ncell, 128), 128, 0, st>>>(G, wrule, ty, tyr, want0, want1, cnt, don, wgt, scal);
  int orphan = kNoOrphan;
  if (hipMemcpyAsync(&orphan, scal, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess || hipGetLastError() != hipSuccess) {
    msg = "assembly kernels failed";
    return UGKS_E_DEVICE;
  }
  if (orphan != kNoOrphan) {
    msg = "overset cell " + std::to_string(orphan) + " has no donor";
    return UGKS_E_ORPHAN;
  }
  // 5. rows in the host order
  const int nrec = scan(want0, nullptr, row0, ncell, 0, sums, scal + 1, st);
  const int nrow = scan(want1, nullptr, row1, ncell, nrec, sums, scal + 1, st);
  const int nd0 = scan(cnt, want0, doff0, ncell, 0, sums, scal + 1, st);
  const int nd = scan(cnt, want1, doff1, ncell, nd0, sums, scal + 1, st);
  if (nrec < 0 || nrow < 0 || nd0 < 0 || nd < 0) {
    msg = "row scan failed";
    return UGKS_E_DEVICE;
  }
  int* drec = S.get<int>(nrow);
  int* dptr = S.get<int>(nrow + 1);
  int* ddon = S.get<int>(nd);
  double* dw = S.get<double>(nd);
  if (!drec || !dptr || !ddon || !dw || hipMemsetAsync(dptr, 0, sizeof(int), st) != hipSuccess) {
    msg = "device allocation failed";
    return UGKS_E_DEVICE;
  }
  k_rows<<<nblk(ncell, 256), 256, 0, st>>>(ncell, want0, want1, row0, row1, doff0, doff1, cnt, don, wgt, drec, dptr,
                                           ddon, dw);
  out.type.resize(ncell);
  out.rec.resize(nrow);
  out.ptr.resize(nrow + 1);
  out.don.resize(nd);
  out.w.resize(nd);
  out.nrec = nrec;
  ok = hipMemcpyAsync(out.type.data(), ty, ncell, hipMemcpyDeviceToHost, st) == hipSuccess &&
       (nrow == 0 || hipMemcpyAsync(out.rec.data(), drec, sizeof(int) * nrow, hipMemcpyDeviceToHost, st) == hipSuccess) &&
       hipMemcpyAsync(out.ptr.data(), dptr, sizeof(int) * (nrow + 1), hipMemcpyDeviceToHost, st) == hipSuccess &&
       (nd == 0 || hipMemcpyAsync(out.don.data(), ddon, sizeof(int) * nd, hipMemcpyDeviceToHost, st) == hipSuccess) &&
       (nd == 0 || hipMemcpyAsync(out.w.data(), dw, sizeof(double) * nd, hipMemcpyDeviceToHost, st) == hipSuccess) &&
       hipStreamSynchronize(st) == hipSuccess && hipGetLastError() == hipSuccess;
  if (!ok) {
    msg = "download of the assembly failed";
    return UGKS_E_DEVICE;
  }
  return UGKS_OK;
}

}  // namespace ugks
