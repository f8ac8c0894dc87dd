// Host launchers of the reverse-mode (adjoint) kernels of libugks; FP64
// storage.  Bars (cotangents) are FP64 device arrays in the layouts of the
// forward arrays; face_bar arrays are [nface][5] = (U_f x, U_f y, wall
// velocity x, y, wall RT).
#pragma once
#include <hip/hip_runtime.h>
#include "ugks_dev.h"

namespace ugks {

// Items (faces, cells or donor rows) grouped by colour: colour i holds
// items[off[i]] .. items[off[i + 1] - 1] (items on the device, off on the
// host).  Items of one colour write disjoint memory in the scatter kernels,
// which run one launch per colour and update with plain read-modify-writes,
// so every bar is summed in an order fixed by the colouring alone and the
// results are bitwise reproducible.
struct Order {
  const int* items = nullptr;
  const int* off = nullptr;
  int ncolour = 0;
};

// workgroups of the face reverse (each strides over its colour's faces and
// stages one face's per-velocity bars in its own [6][nv] slice of fsc)
constexpr int kFaceBlocks = 512;

// UGKS flux (Sec. 2.1) reversed at the state (h, b, W, q) with the cell
// gradients gW of W and the forward face records rec (their moment shifts
// are used): divergence bars Dbh, Dbb [ncell][nv] and face macro flux bar
// Fb [nface][nw] in; bars of h, b, W, q, of gW (scratch, zero on entry) and
// of the face parameters accumulated.  `faces`: the faces that are not
// wall faces, coloured so that a colour's faces touch disjoint cells (both
// sides and the index neighbours of each side); `walls`: the wall faces, a
// colour's faces with disjoint cells and cell neighbours; `cells`: every
// cell, a colour's cells with disjoint sets {c} + nb(c).  fsc: scratch of
// kFaceBlocks x 6 x nv doubles.
void adj_flux(const Dev& g, const Order& faces, const Order& walls, const Order& cells, double dts,
              const double* h, const double* b, const double* W, const double* q, const double* gW,
              const double* rec, const double* Dbh, const double* Dbb, const double* Fb, double* hbar, double* bbar,
              double* Wbar, double* qbar, double* gWbar, double* fbar, double* fsc, hipStream_t st);

// Step 7 and the heat flux of the new state reversed: hb, bb (bars of f')
// updated in place, Wpb = bar of the macro predictor (written)
void adj_step7(const Dev& g, const double* h1, const double* b1, const double* W1, const double* Wp,
               const double* W1b, const double* q1b, double* hb, double* bb, double* Wpb, hipStream_t st);

// micro LU-SGS reversed: x bars (xbh, xbb) in; y, r scratch; sbar scratch
// [ncell][4][2] (face-velocity bars per cell side); bars of f, S, the
// divergence (written), of W~ and of the faces (accumulated)
void adj_micro(const Dev& g, const int* binfo, int nblock, double dt, const double* crec, const double* Wp,
               const double* h0, const double* b0, const double* h1, const double* b1, const double* xsh,
               const double* xsb, const double* xbh, const double* xbb, double* yh, double* yb, double* rh,
               double* rb, double* hbar, double* bbar, double* Shb, double* Sbb, double* Dbh, double* Dbb,
               double* Wpb, double* sbar, double* fbar, hipStream_t st);

// macro LU-SGS reversed: Wpb in; dWb, abar, bbarm, dWsb, Rb scratch; Dgb,
// gamb scratch zero on entry; bars of W, Wn, F, Fn and faces accumulated;
// `faces`, `walls` as for adj_flux
void adj_macro(const Dev& g, const Order& faces, const Order& walls, const int* binfo, int nblock, double dt,
               const double* W, const double* dWs, const double* dW, const double* gam, const double* Wpb,
               double* dWb, double* abar, double* bbarm, double* dWsb, double* Rb, double* Dgb, double* gamb,
               double* Wbar, double* Wnb, double* Fbar, double* Fnb, double* fbar, hipStream_t st);

// Steps 1-2 source reversed: S bars in; bars of f accumulated, divergence
// bars written, bars of W and q accumulated
void adj_source(const Dev& g, double dt, const double* crec, const double* W, const double* h, const double* b,
                const double* Shb, const double* Sbb, double* hbar, double* bbar, double* Dbh, double* Dbb,
                double* Wbar, double* qbar, hipStream_t st);

// overset interpolation reversed for the rows of a donor table (rec, ptr
// start at the first row; `rows` holds row numbers from there, a colour's
// rows with disjoint sets of target and donors)
void adj_interp(const Dev& g, const Order& rows, const int* rec, const int* ptr, const int* don, const double* w,
                double* hbar, double* bbar, double* Wbar, double* qbar, hipStream_t st);

}  // namespace ugks
