// Host-callable launchers of the gfx950 kernels (kernels.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "device.h"

namespace mgc {

// Grid size of the grid-stride vector kernels (dots, axpys, copies).
constexpr int VEC_BLOCKS = 512;

// Optional in-kernel completion of a stencil partial-sum reduction: the last
// block sums the partials into out[0..1] and optionally copies out[0].
// Optional second reduction stage after a stencil pass: out[0..1] = the
// per-block partials added up, out[0] also copied to copy_to (nullable).
struct Finish {
  double* out = nullptr;
  double* copy_to = nullptr;
};

// Scratch of one CCCS application (device pointers, precision-agnostic).
struct CccsScratch {
  void* partA;   // [tiles][n+1][M]  row-projection partials
  void* partB;   // [tiles][n+1][L]  column-projection partials
  void* rhoA;    // [n+1][M]
  void* rhoB;    // [n+1][L]
  void* partC;   // [tiles][M][L]    coupling-coefficient partials
  void* gA;      // [N][M]   local solutions
  void* gB;      // [N][L]
  void* YA;      // [P-1][2M] interface solution
  void* YB;      // [P-1][2L]
  void* HA;      // [P-1][2][2M] halves of the interface right-hand sides
  void* HB;      // [P-1][2][2L]
  void* eA;      // [n+1][M] channel corrections
  void* eB;      // [n+1][L]
};

// Device-resident FGMRES bookkeeping (all pointers into the workspace).
struct GmresState {
  double* hcol;    // [2*(m+1)]     accumulated projections of the current column
  double* nrm2;    // [1]           squared norm
  double* scale;   // [m+2]         1/||W_i|| of the unscaled basis
  double* H;       // [2*(m+1)*m]   Hessenberg, column-major, rotated in place
  double* cs;      // [2*m]
  double* sn;      // [2*m]
  double* g;       // [2*(m+1)]
  double* est;     // [m]           residual estimate after each step
  double* y;       // [2*m]
  double2* upcoef; // [m]           update coefficients y_i
  double* beta;    // [1]
  int* kstar;      // [1]           first step meeting the tolerance (-1: none)
  int* kused;      // [1]
  unsigned* ticket;  // [1]         blocks done in k_reorth_step's second sweep (0 between launches)
};

int launch_stencil_blocks(int n);
int launch_vec_blocks(int n);

template <typename T, typename TU, typename TF, typename TO>
void launch_stencil(hipStream_t s, const Level<T>& L, const void* u, const void* f, void* out,
                    int mode, double* part, Finish fin = Finish());
template <typename T>
void launch_jacobi(hipStream_t s, const Level<T>& L, const void* u, const void* f, void* out, double omega);
template <typename T>
void launch_resid_restrict(hipStream_t s, const Level<T>& L, const void* u, const void* f, void* fc,
                           int pitch_c);
template <typename T>
void launch_prolong_add(hipStream_t s, int n, int pitch, void* u, const void* ec, int pitch_c);
template <typename T>
void launch_coarse_solve(hipStream_t s, const double2* Ainv, int nc, int pitch, const void* f, void* u);

// fused zero-guess passes (nu1 = nu2 = 1); fs: optional device scale of f;
// small: the small tiles (16 x 4 coarse points / 64 x 4 nodes) instead of the
// large ones (32 x 8 / 64 x 16)
template <typename T>
void launch_s1_zero(hipStream_t s, const Level<T>& L, const void* f, const double* fs, double omega,
                    void* fc, int pitch_c, bool small);
template <typename T>
void launch_s2_zero(hipStream_t s, const Level<T>& L, const void* f, const double* fs, double omega,
                    const void* ec, int pitch_c, void* u, bool small);
// S1 of levels l and l+1 in one launch (small tiles): f, fs of level l; f1 =
// f of level l+1 (written), f2 = f of level l+2 (written)
template <typename T>
void launch_s1_pair(hipStream_t s, const Level<T>& Lf, const Level<T>& Lc, const void* f, const double* fs,
                    double omega, void* f1, int pitch1, void* f2, int pitch2);
// S2 of levels l+1 and l in one launch (small tiles): f, fs of level l; fc of
// level l+1; ecc = e of level l+2; u = output of level l
template <typename T>
void launch_s2_pair(hipStream_t s, const Level<T>& Lf, const Level<T>& Lc, const void* f, const double* fs,
                    double omega, const void* fc, const void* ecc, int pitch_cc, void* u);
// coarse tail (levels with n <= TAIL_MAX_N whole in LDS; the kernels take up
// to n = 64): down = S1 passes + coarsest solve, up = S2 passes
template <typename T>
void launch_tail(hipStream_t s, const TailArgs<T>& A, bool down);
constexpr int TAIL_MAX_N = 32;
int launch_cccs_reduce_blocks(int n);   // blocks of coupling-coefficient partials
// Timing hook around one kernel of a multi-kernel launcher: fn(ctx, s, 0)
// before and fn(ctx, s, 1) after the kernel selected by kind.
struct MarkHook {
  void (*fn)(void* ctx, hipStream_t s, int end) = nullptr;
  void* ctx = nullptr;
  int kind = 0;                    // launch_cccs: 1 projection pass, 2 chunk chains, 3 expansion
};
template <typename T>
void launch_cccs(hipStream_t s, const Level<T>& L, void* u, const void* f, const double* fs,
                 const ChanTab<T>& ch, const ChanSys<T>& SA, const ChanSys<T>& SB,
                 const CccsScratch& w, const MarkHook* hook = nullptr);

// Arnoldi step j of FGMRES over the FP64 basis W_0..W_{J-1} (J = j+1 <= 16),
// new vector Y = W_{j+1}; part0..part2 hold ARNOLDI_PART doubles each.
//   apply_dot  : Y = A z, per-block dots W^H Y and ||Y||^2                  -> part0
//   axpy_pass  : coefficients from part0, Y -= ..., dots W^H Y, ||Y||^2     -> part1
//   reorth_step: if pass 0 kept less than eta of ||Y|| (selective
//                re-orthogonalisation) coefficients from part1, Y -= ...,
//                ||Y||^2 -> part2; then ||Y|| (from part2, else from pass
//                0's part1), Hessenberg column j and its Givens rotation;
//                after the cycle's last step (j = mm - 1) also the small
//                least-squares solve (kused, y, update coefficients)
constexpr int ARNOLDI_PART = 256 * 33;
template <typename TZ>
void launch_apply_dot(hipStream_t s, const Level<double>& L, const void* z, size_t stride,
                      const double2* W, int J, double2* Y, double* part0);
// Y32 (nullable, both passes): the new vector also written rounded to FP32,
// unscaled, with the FP64 fields' pitch (the FP32 cycle's input of the next step)
void launch_axpy_pass(hipStream_t s, int n, int pitch, size_t stride, const double2* W, int J,
                      double2* Y, float2* Y32, const double* part0, double* part1, const GmresState& st);
void launch_reorth_step(hipStream_t s, int n, int pitch, size_t stride, const double2* W, int J, double2* Y,
                        float2* Y32, const double* part0, const double* part1, double* part2, const GmresState& st, int m,
                        int mm, double tol_abs, double eta);
constexpr double REORTH_ETA = 0.05;     // default eta
template <typename TZ>
void launch_update(hipStream_t s, int n, int pitch, size_t stride, const void* Z, int J,
                   const double2* coef, double2* u);
template <typename TI, typename TO>
void launch_scale_copy(hipStream_t s, int n, int pitch_in, int pitch_out, const void* in,
                       const double* sc, void* out);
void launch_weight(hipStream_t s, int n, int pitch, const double2* w, int divide, const double2* in,
                   double2* out);
void launch_sum_partials(hipStream_t s, int nb, int nq, const double* part, double* out);
void launch_gmres_begin(hipStream_t s, const GmresState& st, int m);
void launch_ir_scale(hipStream_t s, const double* nrm2, double Nn, double* sc);
void launch_copy_scalar(hipStream_t s, const double* src, double* dst);
// End of a restart cycle: the residual pass's per-block partials (two sums
// over launch_stencil_blocks(n) blocks) into scal[0..1] = (||r||^2, ||f||^2)
// and st.nrm2, the report rep[0..2] = (||r||^2, ||f||^2, kused), then the
// next cycle's start (as launch_gmres_begin).  rep: device memory.
void launch_cycle_end(hipStream_t s, int n, const double* part, double* scal, const GmresState& st, int m,
                      double* rep);
void launch_fill_zero(hipStream_t s, void* p, size_t bytes);   // bytes: multiple of 16
void launch_rhs_tp(hipStream_t s, int n, int pitch, int j0, const double2* z, double Z1, double Z2,
                   double lam, double k0, double2* chi);
void launch_adj_rhs(hipStream_t s, int n, int pitch, int j0, const double2* tm, const double* f1,
                    const double* f2, double2* out);
// VEC_BLOCKS x 12 partials: explicit and adjoint parts of d zeta / d(Z1, Z2, lambda)
void launch_sens_part(hipStream_t s, int n, int pitch, int j0, const double2* z, const double2* tm,
                      const double* f1, const double* f2, const double* df1, const double* df2,
                      const double2* u, const double2* v, const double2* chi, double Z1, double Z2,
                      double lam, double E, double* part);
void launch_zeta_part(hipStream_t s, int n, int pitch, int j0, const double2* tm, const double* f1,
                      const double* f2, const double2* u, const double2* chi, double* part);
// zeta for pp momentum pairs (pp a multiple of 64, <= 256): F1T, F2T are the
// weighted test functions as [n+1][pp] (row = node, column = pair), rows
// 1 .. top of the real region are summed.  part: zeta_sweep_blocks(top) x 2pp
// doubles; out: 2pp doubles (re, im per pair).
int zeta_sweep_blocks(int top);
// The sweep's weighted test functions on the device: F is [2][n+1][pp]
// (x1 side with momenta kk[0 .. npairs), x2 side with kk[npairs .. 2 npairs)),
// zero for the padding pairs npairs .. pp - 1; V1r[j]: the one-body potential
// at the real node x_j = j h.  Needs 1 <= j0 and n >= 2.
void launch_sweep_testfn(hipStream_t s, int n, int j0, double h, const double* V1r, int npairs, int pp,
                         const double* kk, double* F);
// out = chi - v12 u (FP64 fields, interior nodes)
void launch_src_v12(hipStream_t s, int n, int pitch, const double2* chi, const double2* v12, const double2* u,
                    double2* out);
// One GMRES(3) smoothing step on a level (Sec. 6.1): u += V y minimising
// ||f - A(u + V y)|| over K_3(A, f - A u).  V: 4 level fields `stride`
// elements apart; st: 32 doubles of state; part: gmres3_part_doubles(n).
template <typename T>
void launch_gmres3_smooth(hipStream_t s, const Level<T>& L, void* u, const void* f, void* V, size_t stride, double* st,
                          double* part);
int gmres3_part_doubles(int n);
// the V-cycle below and including a GMRES(3) level with n <= GT_MAX_N, in
// one single-workgroup launch
template <typename T>
void launch_gs_tail(hipStream_t s, const GsTailArgs<T>& A);
// u += e on the interior of a level-0 field
template <typename T>
void launch_add(hipStream_t s, int n, int pitch, const void* e, void* u);
// BiCGSTAB (see kernels.hip): bs = device scalar state (11 doubles); the
// partial buffers hold at most 3 x 512 doubles.
void launch_bicg_init(hipStream_t s, double* bs, const double* nrm2);
// p32 / s32 (nullable): the new p / s also written rounded to FP32 (the FP32
// cycle's input), with the FP64 fields' pitch
void launch_bicg_p(hipStream_t s, int n, int pitch, const double2* r, const double2* v, double2* p,
                   float2* p32, const double* bs);
void launch_bicg_s(hipStream_t s, int n, int pitch, const double* part_ad, double* bs, const double2* r,
                   const double2* v, double2* sv, float2* s32, double* part_s);
template <typename TZ>
void launch_bicg_x(hipStream_t s, int n, int pitch, const double* part_ad, const double* part_s, double tol2,
                   double* bs, const void* ph, const void* sh, const double2* sv, const double2* t, const double2* rt,
                   double2* r, double2* x, double* part_x);
void launch_bicg_rho(hipStream_t s, int n, const double* part_x, double* bs, double* rep);
// The x2 side of the single-ionisation sweep from the bound states tab
// ([state][n+1] complex): F2[k][2q] = t_k Re tab_q(k), F2[k][2q+1] = t_k Im
// tab_q(k) on rows 1 .. top, zero elsewhere and for pairs >= 2 nstates.
void launch_bound_weights(hipStream_t s, int n, int top, int j0, double h, int nstates, int pp, const double2* tab,
                          double* F2);
void launch_zeta_sweep(hipStream_t s, int n, int pitch, int top, int pp, const double2* tm, const double* F1T,
                       const double* F2T, const double2* u, const double2* chi, double* part, double* out);

}  // namespace mgc
