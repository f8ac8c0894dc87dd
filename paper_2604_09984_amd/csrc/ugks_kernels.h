// Host-side launchers of the libugks kernels.
#pragma once
#include "ugks_dev.h"

namespace ugks {

// sets the kernels' dynamic LDS limits on the current device; 0 on success
int init_kernel_attributes();
void micro_shape(int dim, int max_ni, int max_nj, int any_pj, int kc_max, int& kc, int& rows);
// the micro sweep's launch for these limits: chunk width, rows per thread,
// register-ring depth and whether the residual is fused into the forward
// sweep (kc = 0 when no shape fits)
void micro_launch_shape(int dim, int prec, int max_ni, int max_nj, int any_pj, int kc_max, int& kc, int& rows,
                        int& depth, int& fused);
size_t micro_lds(int dim, int max_ni, int max_nj, int any_pj, int kc_max);
size_t macro_lds(int nt, int max_ni, int max_nj, int any_pi, int any_pj);

// with ev, four events are recorded: after the wall preparation, after the
// face-moment pass, after its finalize, after the flux pass
void launch_flux(const Dev& g, int prec, const int* binfo, int max_nj, double dts, const void* h, const void* b,
                 const double* W, const double* q, double* gW, double* rec, double* part, void* Dh, void* Db,
                 double* F, double* wall, hipStream_t st, hipEvent_t* ev = nullptr);
// doubles of the per-chunk partial-sum scratch of the flux
inline size_t flux_part_doubles(int nv, int nface) { return (size_t)((nv + 63) / 64) * (size_t)nface * 9; }
void launch_moments(const Dev& g, int prec, const void* h, const void* b, double* W, double* q, hipStream_t st);
void launch_maxwellian(const Dev& g, int prec, const double* W, void* h, void* b, hipStream_t st);
void launch_interp(const Dev& g, int prec, int nrec, const int* rec, const int* ptr, const int* don,
                   const double* w, void* h, void* b, double* W, double* q, hipStream_t st);
void launch_cellrec(const Dev& g, double dt, const double* W, const double* q, const double* mrec, double* crec,
                    hipStream_t st);
void launch_source(const Dev& g, int prec, double dt, const void* h, const void* b, const double* crec,
                   void* Sh, void* Sb, hipStream_t st);
void launch_step7(const Dev& g, int prec, int mode, const void* h, const void* b, const double* crec,
                  const double* Wp, double* W, double* q, double* mrec, hipStream_t st);
void launch_macro(const Dev& g, const int* binfo, int max_ni, int max_nj, int any_pi, int any_pj, double dt,
                  const double* W, const double* Wn, const double* F, const double* Fn, double* gam, double* R,
                  double* Dg, double* dWs, double* dW, double* Wp, double* rpart, double* resid, hipStream_t st);
void launch_micro(const Dev& g, int prec, const int* binfo, int max_ni, int max_nj, int any_pj, double dt,
                  const double* crec, void* h, void* b, const void* Sh, const void* Sb, void* Dh, void* Db,
                  hipStream_t st, hipEvent_t* ev = nullptr);

// ---------------------------------------------------------------------------
// Batched pseudo-iteration: many cases advanced by one launch per stage.
// Each case's arguments live in a device table; the per-cell and per-face
// stages run one flat grid whose workgroups find their case in a prefix
// table of per-case workgroup counts; the march passes and the micro sweep
// are persistent grids striding over (case, velocity chunk, row group,
// block) work items, ordered by decreasing cost.  Every work item runs the
// same code as the case's own launch, so each case's results are those of
// its own pseudo-iteration, bit for bit.
struct BatchCase {
  Dev g;
  const int* binfo;
  int nchunk, nrec;
  double dt, dts;
  void *h, *b, *Dh, *Db;
  const void *Sh, *Sb;
  double *W, *q, *resid;
  const double *Wn, *Fn;
  double *gW, *rec, *part, *F, *gam, *mac, *dWs, *dW, *Wp, *rpart, *crec, *mrec;
  const int *orec, *optr, *odon;
  const double* ow;
};
struct BatchItem {
  int cs, x, y, z;  // case; chunk; row group (march) or block (micro); block (march)
};
struct BatchPlan {
  int ncase = 0, prec = 0;
  const BatchCase* cases = nullptr;  // device [ncase]
  // device prefix tables [ncase + 1] of per-case workgroup counts and their
  // totals: 64-thread workgroups over cells and faces, 4 cells or receptors
  // per 256-thread workgroup, one per block, one per case
  const int *off_cell64 = nullptr, *off_face64 = nullptr, *off_cell4 = nullptr, *off_rec4 = nullptr,
            *off_block = nullptr;
  int n_cell64 = 0, n_face64 = 0, n_cell4 = 0, n_rec4 = 0, n_block = 0;
  // work items of the face-moment [0] and flux [1] march passes (rg[m] core
  // rows per workgroup) and of the micro sweep (device)
  const BatchItem* march_items[2] = {nullptr, nullptr};
  const BatchItem* micro_items = nullptr;
  int n_march[2] = {0, 0}, grid_march[2] = {0, 0}, rg[2] = {8, 8};
  int n_micro = 0, grid_micro = 0;
  // launch shapes common to the batch
  int micro_kc = 0, micro_rows = 1, micro_nslot = 0, macro_nt = 64;
  size_t micro_lds = 0, macro_lds = 0;
  int max_ni = 0, max_nj = 0, any_pi = 0, any_pj = 0;
  int want_resid = 0;
};
// persistent grid sizes (host): of a march pass (mode 0 face moments, 1
// flux) with rg core rows per workgroup, and of the micro sweep with its LDS
int batch_march_grid(int prec, int rg, int mode, int& grid);
int batch_micro_grid(size_t micro_lds, int& grid);
// the pseudo-iterations of a batch (2D, one storage type) on stream st
void launch_batch_inner(const BatchPlan& p, int n_inner, hipStream_t st);

// fills n doubles with v (a kernel, so that captured graphs hold no memset)
void launch_fill(double* a, size_t n, double v, hipStream_t st);
// wall loads from a face macro flux F: face_out [nface][dim+3] (zero off the
// walls), side_out [nside][4]; either may be null
void launch_wall_loads(const Dev& g, int nside, const int* wptr, const double* wtab, const double* F,
                       double* face_out, double* side_out, hipStream_t st);
// F_bar [nface][nw] (written) from the cotangents of the wall loads
void launch_wall_loads_adj(const Dev& g, int nside, const int* wptr, const double* wtab, const double* face_bar,
                           const double* side_bar, double* F_bar, hipStream_t st);
// U_bar [nblock][2], rtw_bar [nblock][4] from per-face cotangents [nface][5]
void launch_param_bars(int nblock, const int* bface, const int* wptr, const double* wtab, const double* face_bar,
                       double* U_bar, double* rtw_bar, hipStream_t st);

// The scratch array of the entry points that allocate nothing: a file-scope
// device array of kStaticScratchBytes, one per device.  Sets *ptr to this
// device's address of it (looked up once per device, with that device
// current, then cached); 0 on success.
constexpr size_t kStaticScratchBytes = (size_t)128 << 20;
int static_scratch(int device, void** ptr);

}  // namespace ugks
