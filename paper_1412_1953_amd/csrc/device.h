// Device-side types shared by the HIP kernels and the host launch code.
#pragma once
#include <hip/hip_runtime.h>

namespace mgc {

template <typename T> struct vec2;
template <> struct vec2<double> { using type = double2; };
template <> struct vec2<float> { using type = float2; };
template <typename T> using v2 = typename vec2<T>::type;

// One multigrid level as seen by a stencil kernel.  All tables have n+1
// entries indexed by node; entries 0 and n are never used.
//   a, c : 3-point coefficients of -1/2 d^2/dz^2 (sub / super)
//   px   : b_j + V1_j   (x1 diagonal part)
//   py   : b_k + V2_k   (x2 diagonal part)
//   tm   : lambda / z_m (two-body part, evaluated at m = max(j,k))
//   v12  : null, or a general two-body potential V12(z_j, z_k) as a field
//          ((n+1) rows x pitch, same layout as the unknowns)
// Diagonal of the operator: px[j] + py[k] + tm[max(j,k)] (+ v12[k][j]) - E.
template <typename T> struct Level {
  const v2<T>* a;
  const v2<T>* c;
  const v2<T>* px;
  const v2<T>* py;
  const v2<T>* tm;
  const v2<T>* v12;
  int n;
  int pitch;
  T E;
};

// Coarse tail of the zero-guess V-cycle: smoothing levels lt .. lt+nl-1 (each
// with n <= 64) and the coarsest level lt+nl, indexed from 0 here.
constexpr int TMAXL = 4;
template <typename T> struct TailArgs {
  Level<T> L[TMAXL];          // smoothing levels
  v2<T>* f[TMAXL + 1];        // f[0]: input; f[1..nl]: restricted residuals
  v2<T>* u[TMAXL + 1];        // u[0]: output; u[nl]: coarsest solution
  int pitch[TMAXL + 1];
  int nl;                     // number of smoothing levels, 1..TMAXL
  int nc;                     // n of the coarsest level
  const double2* Ainv;        // dense inverse on the coarsest level
  const double* fs;           // optional device scale of f[0]
  T omega;
};

// Coarse tail of a V-cycle whose levels all take the GMRES(3) smoother: the
// levels lt .. lt+nl-1 (n <= GT_MAX_N, finest first) and the coarsest level,
// run by one workgroup (k_gs_tail).
constexpr int GT_MAX_N = 64;
template <typename T> struct GsTailArgs {
  Level<T> L[TMAXL];          // smoothing levels
  const v2<T>* f0;            // right-hand side of the top level
  v2<T>* u0;                  // iterate of the top level (in: unless zero; out)
  v2<T>* f[TMAXL + 1];        // f[1..nl]: restricted right-hand sides
  v2<T>* u[TMAXL + 1];        // u[1..nl-1]: iterates between the passes
  int pitch[TMAXL + 1];
  int nl;                     // number of smoothing levels, 1..TMAXL
  int nc;                     // n of the coarsest level
  const double2* Ainv;        // dense inverse on the coarsest level
  int zero;                   // the top level starts from u = 0
  int nu1, nu2;
};

// CCCS tables of one precision on level 0.
template <typename T> struct ChanTab {
  const v2<T>* wphi;   // [M][n+1]  w_j phi_i(z_j)       (x1 channels)
  const v2<T>* phi;    // [M][n+1]  phi_i(z_j)
  const v2<T>* wvphi;  // [L][n+1]  w_k varphi_l(z_k)    (x2 channels)
  const v2<T>* vphi;   // [L][n+1]  varphi_l(z_k)
  int M, L;
};

// Factors of one coupled channel system (see ChannelFactors on the host).
template <typename T> struct ChanSys {
  const v2<T>* G;      // [N][M][M]
  const v2<T>* Vs;     // [N][M][M]
  const v2<T>* Ws;     // [N][M][M]
  const v2<T>* lo;     // [N]
  const v2<T>* up;     // [N]
  const v2<T>* Rinv;   // [P-1][2M][2M]
  const v2<T>* Tif;    // [(P-1)2M][(P-1)2M] interface solve as one matrix
  const int* start;    // [P+1]
  int N, M, P;
};

}  // namespace mgc
