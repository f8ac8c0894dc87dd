// Host launchers of the reverse-mode (adjoint) kernels of libugks; FP64
// storage.  Bars (cotangents) are FP64 device arrays in the layouts of the
// forward arrays; face_bar arrays are [nface][5] = (U_f x, U_f y, wall
// velocity x, y, wall RT).
#pragma once
#include <hip/hip_runtime.h>
#include "ugks_dev.h"

namespace ugks {

// UGKS flux (Sec. 2.1) reversed at the state (h, b, W, q) with the cell
// gradients gW of W and the forward face records rec (their moment shifts
// are used): divergence bars Dbh, Dbb [ncell][nv] and face macro flux bar
// Fb [nface][nw] in; bars of h, b, W, q, of gW (scratch, zero on entry) and
// of the face parameters accumulated.
void adj_flux(const Dev& g, double dts, const double* h, const double* b, const double* W, const double* q,
              const double* gW, const double* rec, const double* Dbh, const double* Dbb, const double* Fb,
              double* hbar, double* bbar, double* Wbar, double* qbar, double* gWbar, double* fbar, hipStream_t st);

// Step 7 and the heat flux of the new state reversed: hb, bb (bars of f')
// updated in place, Wpb = bar of the macro predictor (written)
void adj_step7(const Dev& g, const double* h1, const double* b1, const double* W1, const double* Wp,
               const double* W1b, const double* q1b, double* hb, double* bb, double* Wpb, hipStream_t st);

// micro LU-SGS reversed: x bars (xbh, xbb) in; y, r scratch; bars of f,
// S, the divergence (written), of W~ and of the faces (accumulated)
void adj_micro(const Dev& g, const int* binfo, int nblock, double dt, const double* crec, const double* Wp,
               const double* h0, const double* b0, const double* h1, const double* b1, const double* xsh,
               const double* xsb, const double* xbh, const double* xbb, double* yh, double* yb, double* rh,
               double* rb, double* hbar, double* bbar, double* Shb, double* Sbb, double* Dbh, double* Dbb,
               double* Wpb, double* fbar, hipStream_t st);

// macro LU-SGS reversed: Wpb in; dWb, abar, bbarm, dWsb, Rb scratch; Dgb,
// gamb scratch zero on entry; bars of W, Wn, F, Fn and faces accumulated
void adj_macro(const Dev& g, const int* binfo, int nblock, double dt, const double* W, const double* dWs,
               const double* dW, const double* gam, const double* Wpb, double* dWb, double* abar, double* bbarm,
               double* dWsb, double* Rb, double* Dgb, double* gamb, double* Wbar, double* Wnb, double* Fbar,
               double* Fnb, double* fbar, hipStream_t st);

// Steps 1-2 source reversed: S bars in; bars of f accumulated, divergence
// bars written, bars of W and q accumulated
void adj_source(const Dev& g, double dt, const double* crec, const double* W, const double* h, const double* b,
                const double* Shb, const double* Sbb, double* hbar, double* bbar, double* Dbh, double* Dbb,
                double* Wbar, double* qbar, hipStream_t st);

// overset interpolation reversed for nrow rows of a donor table
void adj_interp(const Dev& g, int nrow, const int* rec, const int* ptr, const int* don, const double* w,
                double* hbar, double* bbar, double* Wbar, double* qbar, hipStream_t st);

}  // namespace ugks
