// gfx950 kernels of the MG-CCCS solver.
//
// Field layout: (n+1) rows x pitch columns of interleaved complex values, row
// k along x2, column j along x1 (contiguous).  Interior nodes 1..n-1 in both
// directions; the Dirichlet ring is treated as zero by index tests and is
// never written.  Every kernel bounds-checks its node against [1, n-1].
//
// Reductions are deterministic: per-block partial sums in a fixed order
// (wave shuffles, then LDS), then a second single-block pass.  No floating
// point atomics are used anywhere.
#include <algorithm>

#include "device.h"
#include "launch.h"

namespace mgc {

// ----------------------------------------------------------------------------
// complex helpers.  The library is built without implicit contraction, so a
// product meets an add in one rounding only where an fma is written out here:
// every kernel that evaluates one of these operations rounds it the same way.
template <typename T> __device__ __forceinline__ v2<T> mk(T x, T y) { v2<T> r; r.x = x; r.y = y; return r; }
__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
// 1 / x for the complex divisions by an operator diagonal (x = |d|^2 > 0, far
// from the underflow and overflow ranges).  FP64: the hardware reciprocal
// estimate refined by two Newton steps r <- r + r (1 - x r), within an ulp or
// so of the correctly rounded quotient at a third of the instructions of an
// IEEE division; FP32 keeps the IEEE quotient.  One definition for every
// kernel, so that each evaluation of a division rounds the same way.
__device__ __forceinline__ double recipT(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fmaT(r, fmaT(-x, r, 1.0), r);
  return fmaT(r, fmaT(-x, r, 1.0), r);
}
__device__ __forceinline__ float recipT(float x) { return 1.0f / x; }
#define MGC_CPLX_OPS(V, T)                                                                  \
  __device__ __forceinline__ V cadd(V a, V b) { return mk<T>(a.x + b.x, a.y + b.y); }        \
  __device__ __forceinline__ V csub(V a, V b) { return mk<T>(a.x - b.x, a.y - b.y); }        \
  __device__ __forceinline__ V cmul(V a, V b) {                                             \
    return mk<T>(fmaT(a.x, b.x, -(a.y * b.y)), fmaT(a.x, b.y, a.y * b.x));                  \
  }                                                                                         \
  /* acc + a*b */                                                                           \
  __device__ __forceinline__ V cfma(V acc, V a, V b) {                                      \
    return mk<T>(fmaT(a.x, b.x, fmaT(-a.y, b.y, acc.x)), fmaT(a.x, b.y, fmaT(a.y, b.x, acc.y))); \
  }                                                                                         \
  __device__ __forceinline__ V cscale(V a, T s) { return mk<T>(a.x * s, a.y * s); }          \
  /* |b|^2 */                                                                               \
  __device__ __forceinline__ T cabs2(V b) { return fmaT(b.x, b.x, b.y * b.y); }              \
  __device__ __forceinline__ V cdiv(V a, V b) {                                             \
    T inv = recipT(cabs2(b));                                                               \
    return mk<T>(fmaT(a.x, b.x, a.y * b.y) * inv, fmaT(a.y, b.x, -(a.x * b.y)) * inv);      \
  }                                                                                         \
  /* a / b with inv = recipT(|b|^2) given (the same arithmetic as cdiv) */                      \
  __device__ __forceinline__ V cdiv_inv(V a, V b, T inv) {                                  \
    return mk<T>(fmaT(a.x, b.x, a.y * b.y) * inv, fmaT(a.y, b.x, -(a.x * b.y)) * inv);      \
  }
MGC_CPLX_OPS(double2, double)
MGC_CPLX_OPS(float2, float)
#undef MGC_CPLX_OPS
template <typename T, typename V> __device__ __forceinline__ v2<T> cvt(V v) {
  return mk<T>((T)v.x, (T)v.y);
}
template <typename T, typename V>
__device__ __forceinline__ v2<T> ldf(const V* p, int pitch, int k, int j, int n) {
  if (j <= 0 || j >= n || k <= 0 || k >= n) return mk<T>(0, 0);
  return cvt<T>(p[(size_t)k * pitch + j]);
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// General two-body table at node (k, j), the indices clamped onto the grid
// (nodes outside it only occur in halos whose values are never used)
template <typename T>
__device__ __forceinline__ v2<T> v12_at(const Level<T>& L, int k, int j) {
  const int kk = k < 0 ? 0 : (k > L.n ? L.n : k), jj = j < 0 ? 0 : (j > L.n ? L.n : j);
  return L.v12[(size_t)kk * L.pitch + jj];
}

// Operator diagonal at (k, j): px_j + py_k + tm_max(j,k) (+ v12_kj) - E
template <typename T>
__device__ __forceinline__ v2<T> diag_at(const Level<T>& L, int k, int j) {
  v2<T> d = cadd(cadd(L.px[j], L.py[k]), L.tm[j > k ? j : k]);
  if (L.v12) d = cadd(d, v12_at(L, k, j));
  d.x -= L.E;
  return d;
}

// (A u)(k, j) for an interior node
template <typename T, typename VU>
__device__ __forceinline__ v2<T> apply_at(const Level<T>& L, const VU* u, int k, int j) {
  const int n = L.n, p = L.pitch;
  v2<T> uc = ldf<T>(u, p, k, j, n);
  v2<T> acc = cmul(diag_at(L, k, j), uc);
  acc = cfma(acc, L.a[j], ldf<T>(u, p, k, j - 1, n));
  acc = cfma(acc, L.c[j], ldf<T>(u, p, k, j + 1, n));
  acc = cfma(acc, L.a[k], ldf<T>(u, p, k - 1, j, n));
  acc = cfma(acc, L.c[k], ldf<T>(u, p, k + 1, j, n));
  return acc;
}


// Column-resident 5-point stencil for a thread that walks down one column j:
// keeps u(k-1, j), u(k, j) in registers (one new load per row) and the x1
// tables of its column; the x2 tables of the current row are wave-uniform.
template <typename T, typename VU>
struct ColumnStencil {
  const Level<T>& L;
  const VU* u;
  int j;
  v2<T> aj, cj, pxj, um, uc;
  __device__ ColumnStencil(const Level<T>& L_, const VU* u_, int j_, int k0)
      : L(L_), u(u_), j(j_) {
    const bool ok = j > 0 && j < L.n;
    aj = ok ? L.a[j] : mk<T>(0, 0);
    cj = ok ? L.c[j] : mk<T>(0, 0);
    pxj = ok ? L.px[j] : mk<T>(0, 0);
    um = ldf<T>(u, L.pitch, k0 - 1, j, L.n);
    uc = ldf<T>(u, L.pitch, k0, j, L.n);
  }
  // (A u)(k, j) for k = current row; then advance to row k+1
  __device__ __forceinline__ v2<T> step(int k) {
    const int n = L.n, p = L.pitch;
    const v2<T> up = ldf<T>(u, p, k + 1, j, n);
    if (j <= 0 || j >= n) {          // column outside the grid: no table access
      um = uc;
      uc = up;
      return mk<T>(0, 0);
    }
    const v2<T> uw = ldf<T>(u, p, k, j - 1, n), ue = ldf<T>(u, p, k, j + 1, n);
    v2<T> d = cadd(cadd(pxj, L.py[k]), L.tm[j > k ? j : k]);
    if (L.v12) d = cadd(d, v12_at(L, k, j));
    d.x -= L.E;
    v2<T> acc = cmul(d, uc);
    acc = cfma(acc, aj, uw);
    acc = cfma(acc, cj, ue);
    acc = cfma(acc, L.a[k], um);
    acc = cfma(acc, L.c[k], up);
    um = uc;
    uc = up;
    return acc;
  }
};

// Block-level reduction of NV doubles held per thread; thread 0 of the block
// ends with the totals in out[].  blockDim.x * blockDim.y must be a multiple
// of 64 and at most 1024.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* out) {
  __shared__ double red[16][NV];
  const int tid = threadIdx.x + blockDim.x * threadIdx.y;
  const int lane = tid & 63, wid = tid >> 6, nw = (blockDim.x * blockDim.y) >> 6;
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] = wave_sum(v[q]);
  if (lane == 0)
#pragma unroll
    for (int q = 0; q < NV; ++q) red[wid][q] = v[q];
  __syncthreads();
  if (tid == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      double s = 0;
      for (int w = 0; w < nw; ++w) s += red[w][q];
      out[q] = s;
    }
  }
  __syncthreads();
}

// Second stage of a two-stage reduction on partials written by an earlier
// kernel, run by one block of NT threads: out[q] = sum_b part[b*stride + q]
// (stride defaults to nq; nq <= NT).  Thread slice sl sums b = sl, sl + ns, ...
// in groups of eight loads issued together (pairwise within a group, groups in
// ascending order); the slices are then combined in ascending order.  The
// order depends only on (nb, nq, NT).  Ends with a barrier.
template <int NT>
__device__ __forceinline__ double slice_sum(const double* part, int nb, int stride, int q, int sl, int ns) {
  double s = 0.0;
  for (int b0 = sl; b0 < nb; b0 += 8 * ns) {
    double v[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int b = b0 + i * ns;
      v[i] = b < nb ? part[(size_t)b * stride + q] : 0.0;
    }
    s += ((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]));
  }
  return s;
}
template <int NT>
__device__ void finish_sum_nt(const double* part, int nb, int nq, double* out, int stride = 0) {
  if (stride == 0) stride = nq;
  __shared__ double red[NT];
  const int t = threadIdx.x + blockDim.x * threadIdx.y;
  const int ns = NT / nq;
  const int q = t % nq, sl = t / nq;
  red[t] = sl < ns ? slice_sum<NT>(part, nb, stride, q, sl, ns) : 0.0;
  __syncthreads();
  if (t < nq) {
    double tot = 0.0;
    for (int w = 0; w < ns; ++w) tot += red[w * nq + t];
    out[t] = tot;
  }
  __syncthreads();
}
__device__ void finish_sum(const double* part, int nb, int nq, double* out) {
  finish_sum_nt<256>(part, nb, nq, out);
}
// Two single sums in one pass (half of the block each):
// out[0] = sum_b a[b*sa], out[1] = sum_b c[b*sc].  Each thread sums its slice,
// the waves reduce by shuffles, the per-wave sums are added in wave order.
// Ends with a barrier.
template <int NT>
__device__ void finish_sum_pair(const double* a, int na, int sa, const double* c, int nc, int sc,
                                double* out) {
  static_assert(NT % 128 == 0, "whole waves per half");
  constexpr int H = NT / 2, HW = H / 64;
  __shared__ double red[NT / 64];
  const int t = threadIdx.x + blockDim.x * threadIdx.y;
  double s = t < H ? slice_sum<NT>(a, na, sa, 0, t, H) : slice_sum<NT>(c, nc, sc, 0, t - H, H);
  s = wave_sum(s);
  if ((t & 63) == 0) red[t >> 6] = s;
  __syncthreads();
  if (t < 2) {
    double tot = 0.0;
    for (int w = 0; w < HW; ++w) tot += red[t * HW + w];
    out[t] = tot;
  }
  __syncthreads();
}

// ----------------------------------------------------------------------------
// Stencil kernels: block (64, 4), each thread one column and ROWS rows.
constexpr int SX = 64, SY = 4, ROWS = 4;

// mode 0: out = f - A u ; mode 1: out = A u.  part (nullable): per block
// [sum |out|^2, sum |f|^2] (mode 0) accumulated in FP64.
template <typename T, typename TU, typename TF, typename TO>
__global__ void __launch_bounds__(256) k_stencil(Level<T> L, const v2<TU>* __restrict__ u,
                                                 const v2<TF>* __restrict__ f,
                                                 v2<TO>* __restrict__ out, int mode,
                                                 double* __restrict__ part) {
  const int j = 1 + blockIdx.x * SX + threadIdx.x;
  const int k0 = 1 + (blockIdx.y * SY + threadIdx.y) * ROWS;
  const int n = L.n, p = L.pitch;
  double acc[2] = {0.0, 0.0};
  if (j < n) {
    ColumnStencil<T, v2<TU>> cs(L, u, j, __builtin_amdgcn_readfirstlane(k0));
    for (int r = 0; r < ROWS; ++r) {
      const int k = __builtin_amdgcn_readfirstlane(k0 + r);
      if (k >= n) break;
      v2<T> Au = cs.step(k);
      v2<T> o;
      if (mode == 0) {
        v2<T> fv = cvt<T>(f[(size_t)k * p + j]);
        o = csub(fv, Au);
        acc[1] += (double)fv.x * fv.x + (double)fv.y * fv.y;
      } else {
        o = Au;
      }
      acc[0] += (double)o.x * o.x + (double)o.y * o.y;
      out[(size_t)k * p + j] = cvt<TO>(o);
    }
  }
  if (part) {
    double tot[2];
    block_sum<2>(acc, tot);
    if (threadIdx.x == 0 && threadIdx.y == 0) {
      const int b = blockIdx.x + gridDim.x * blockIdx.y;
      part[2 * b] = tot[0];
      part[2 * b + 1] = tot[1];
    }
  }
}

// omega-Jacobi: out = u + omega (f - A u) / d ; u == nullptr means u = 0.
template <typename T>
__global__ void __launch_bounds__(256) k_jacobi(Level<T> L, const v2<T>* __restrict__ u,
                                                const v2<T>* __restrict__ f,
                                                v2<T>* __restrict__ out, T omega) {
  const int j = 1 + blockIdx.x * SX + threadIdx.x;
  const int k0 = 1 + (blockIdx.y * SY + threadIdx.y) * ROWS;
  const int n = L.n, p = L.pitch;
  if (j >= n) return;
  for (int r = 0; r < ROWS; ++r) {
    const int k = k0 + r;
    if (k >= n) break;
    const size_t idx = (size_t)k * p + j;
    v2<T> fv = f[idx];
    v2<T> d = diag_at(L, k, j);
    v2<T> o;
    if (u) {
      v2<T> res = csub(fv, apply_at<T>(L, u, k, j));
      o = cadd(u[idx], cscale(cdiv(res, d), omega));
    } else {
      o = cscale(cdiv(fv, d), omega);
    }
    out[idx] = o;
  }
}

// Residual + full weighting:  fc(K,J) = (1/16) sum w_ab r(2K+a, 2J+b),
// weights [1 2 1; 2 4 2; 1 2 1], r = f - A u on the fine level.
template <typename T>
__global__ void __launch_bounds__(256) k_resid_restrict(Level<T> L, const v2<T>* __restrict__ u,
                                                        const v2<T>* __restrict__ f,
                                                        v2<T>* __restrict__ fc, int pitch_c) {
  const int nc = L.n / 2;
  const int J = 1 + blockIdx.x * SX + threadIdx.x;
  const int K = 1 + blockIdx.y * SY + threadIdx.y;
  if (J >= nc || K >= nc) return;
  const int p = L.pitch;
  v2<T> acc = mk<T>(0, 0);
#pragma unroll
  for (int a = -1; a <= 1; ++a) {
#pragma unroll
    for (int b = -1; b <= 1; ++b) {
      const int k = 2 * K + a, j = 2 * J + b;
      v2<T> r = csub(cvt<T>(f[(size_t)k * p + j]), apply_at<T>(L, u, k, j));
      const T w = T((a == 0 ? 2 : 1) * (b == 0 ? 2 : 1));
      acc = mk<T>(acc.x + w * r.x, acc.y + w * r.y);
    }
  }
  fc[(size_t)K * pitch_c + J] = cscale(acc, T(1.0 / 16.0));
}

// u += bilinear interpolation of the coarse correction ec.
template <typename T>
__global__ void __launch_bounds__(256) k_prolong_add(int n, int pitch, v2<T>* __restrict__ u,
                                                     const v2<T>* __restrict__ ec, int pitch_c) {
  const int j = 1 + blockIdx.x * SX + threadIdx.x;
  const int k0 = 1 + (blockIdx.y * SY + threadIdx.y) * ROWS;
  if (j >= n) return;
  const int nc = n / 2;
  const int J0 = j >> 1, J1 = (j + 1) >> 1;      // equal for even j
  for (int r = 0; r < ROWS; ++r) {
    const int k = k0 + r;
    if (k >= n) break;
    const int K0 = k >> 1, K1 = (k + 1) >> 1;
    v2<T> s = cadd(cadd(ldf<T>(ec, pitch_c, K0, J0, nc), ldf<T>(ec, pitch_c, K0, J1, nc)),
                   cadd(ldf<T>(ec, pitch_c, K1, J0, nc), ldf<T>(ec, pitch_c, K1, J1, nc)));
    const size_t idx = (size_t)k * pitch + j;
    u[idx] = cadd(u[idx], cscale(s, T(0.25)));
  }
}

// Coarsest level: u = Ainv f with the dense FP64 inverse (row-major, unknown
// index (k-1)*(nc-1) + (j-1)).  One wave per row.
template <typename T>
__global__ void __launch_bounds__(256) k_coarse_solve(const double2* __restrict__ Ainv, int nc,
                                                      int pitch, const v2<T>* __restrict__ f,
                                                      v2<T>* __restrict__ u) {
  const int m = nc - 1, N = m * m;
  const int row = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (row >= N) return;
  double sr = 0, si = 0;
  const double2* Ar = Ainv + (size_t)row * N;
  for (int c = lane; c < N; c += 64) {
    const int k = c / m + 1, j = c % m + 1;
    v2<double> fv = cvt<double>(f[(size_t)k * pitch + j]);
    double2 a = Ar[c];
    sr += a.x * fv.x - a.y * fv.y;
    si += a.x * fv.y + a.y * fv.x;
  }
  sr = wave_sum(sr);
  si = wave_sum(si);
  if (lane == 0) {
    const int k = row / m + 1, j = row % m + 1;
    u[(size_t)k * pitch + j] = mk<T>((T)sr, (T)si);
  }
}


// ----------------------------------------------------------------------------
// Fused zero-guess V-cycle passes (nu1 = nu2 = 1).  With u = 0 on entry the
// pre-smoothed iterate is u' = omega f / d pointwise, so it is never stored:
//   S1: r = f - A u' on the fine tile, then full weighting -> f_c
//   S2: w = u' + P e_c, then one omega-Jacobi sweep -> u
// fs (nullable, device scalar) scales f on the fly.
// S1 tile: CX x CY coarse points per block (32 x 8 on the finest levels,
// 16 x 4 where the large tiles would give fewer than two blocks per CU)
template <int CX_, int CY_> struct S1Tile {
  static constexpr int CX = CX_, CY = CY_;
  static constexpr int W = 2 * CX + 3, H = 2 * CY + 3;     // u' tile (fine nodes)
  static constexpr int RW = 2 * CX + 1, RH = 2 * CY + 1;   // residual region
  static constexpr int NR = (RH * RW + 255) / 256;         // residual points per thread
  static constexpr int NH = (H * W - RH * RW + 255) / 256; // halo points per thread
};
using S1Big = S1Tile<32, 8>;
using S1Small = S1Tile<16, 4>;

// 1D operator tables of a tile, staged in LDS in the same load round as the
// field values: by column (px, a, c, tm at the columns' x1 nodes) and by row
// (py, a, c, tm at the rows' x2 nodes); zero outside the interior.
template <typename T, int W, int H> struct TileTabs {
  v2<T> col[4][W];
  v2<T> row[4][H];
};
template <typename T, int W, int H>
__device__ __forceinline__ void stage_tabs(TileTabs<T, W, H>& tb, const Level<T>& L, int c0, int r0, int tid) {
  if (tid < W + H) {
    const bool isc = tid < W;
    const int ix = isc ? c0 + tid : r0 + (tid - W);
    const bool ok = ix > 0 && ix < L.n;
    const int ic = ok ? ix : 1;
    const v2<T>* pd = isc ? L.px : L.py;
    v2<T> t0 = pd[ic], t1 = L.a[ic], t2 = L.c[ic], t3 = L.tm[ic];
    if (!ok) t0 = t1 = t2 = t3 = mk<T>(0, 0);
    if (isc) {
      tb.col[0][tid] = t0; tb.col[1][tid] = t1; tb.col[2][tid] = t2; tb.col[3][tid] = t3;
    } else {
      const int r = tid - W;
      tb.row[0][r] = t0; tb.row[1][r] = t1; tb.row[2][r] = t2; tb.row[3][r] = t3;
    }
  }
}
// diagonal px_j + py_k + tm_max(j,k) (+ v12_kj) - E at tile position (rr, cc),
// node (k, j) of level L
template <typename T, int W, int H>
__device__ __forceinline__ v2<T> tab_diag(const TileTabs<T, W, H>& tb, const Level<T>& L, int rr, int cc, int k,
                                          int j) {
  v2<T> d = cadd(cadd(tb.col[0][cc], tb.row[0][rr]), j > k ? tb.col[3][cc] : tb.row[3][rr]);
  if (L.v12) d = cadd(d, v12_at(L, k, j));
  d.x -= L.E;
  return d;
}
// (A w)(k, j) from an LDS tile w with a one-node halo; tab_apply_d takes the
// diagonal d at (k, j) already formed
template <typename T, int W, int H, int TW>
__device__ __forceinline__ v2<T> tab_apply_d(const TileTabs<T, W, H>& tb, v2<T> d, const v2<T> (*w)[TW], int rr,
                                             int cc) {
  v2<T> acc = cmul(d, w[rr][cc]);
  acc = cfma(acc, tb.col[1][cc], w[rr][cc - 1]);
  acc = cfma(acc, tb.col[2][cc], w[rr][cc + 1]);
  acc = cfma(acc, tb.row[1][rr], w[rr - 1][cc]);
  acc = cfma(acc, tb.row[2][rr], w[rr + 1][cc]);
  return acc;
}
template <typename T, int W, int H, int TW>
__device__ __forceinline__ v2<T> tab_apply(const TileTabs<T, W, H>& tb, const Level<T>& L, const v2<T> (*w)[TW],
                                           int rr, int cc, int k, int j) {
  v2<T> acc = cmul(tab_diag(tb, L, rr, cc, k, j), w[rr][cc]);
  acc = cfma(acc, tb.col[1][cc], w[rr][cc - 1]);
  acc = cfma(acc, tb.col[2][cc], w[rr][cc + 1]);
  acc = cfma(acc, tb.row[1][rr], w[rr - 1][cc]);
  acc = cfma(acc, tb.row[2][rr], w[rr + 1][cc]);
  return acc;
}

// S1 tile loads: every thread first takes its points of the residual region
// (kept in registers for the residual), then at most one halo point, so that
// only u' needs an LDS tile.
template <typename T, typename TL>
__global__ void __launch_bounds__(256) k_s1_zero(Level<T> L, const v2<T>* __restrict__ f,
                                                 const double* __restrict__ fs, T omega,
                                                 v2<T>* __restrict__ fc, int pitch_c) {
  constexpr int S1CX = TL::CX, S1CY = TL::CY, S1W = TL::W, S1H = TL::H, S1RW = TL::RW, S1RH = TL::RH;
  constexpr int S1NR = TL::NR, S1NH = TL::NH;
  __shared__ v2<T> up[S1H][S1W];          // u', then the residual on the same nodes
  __shared__ TileTabs<T, S1W, S1H> tb;
  const int n = L.n, p = L.pitch, nc = n / 2;
  const int tid = threadIdx.x + 64 * threadIdx.y;
  const int J0 = 1 + blockIdx.x * S1CX, K0 = 1 + blockIdx.y * S1CY;
  const int c0 = 2 * J0 - 2, r0 = 2 * K0 - 2;             // fine origin of the u' tile
  const T sc = fs ? (T)*fs : T(1);
  // tile position of the thread's q-th residual-region point / halo point
  auto rpos = [&](int q, int& rr, int& cc) {
    const int idx = tid + 256 * q;
    rr = 1 + idx / S1RW;
    cc = 1 + idx % S1RW;
    return idx < S1RH * S1RW;
  };
  auto hpos = [&](int q, int& rr, int& cc) {
    const int h = tid + 256 * q;                 // halo: rows 0 and S1H-1, columns 0 and S1W-1
    if (h < S1W) { rr = 0; cc = h; return true; }
    if (h < 2 * S1W) { rr = S1H - 1; cc = h - S1W; return true; }
    const int v = h - 2 * S1W;
    if (v < 2 * (S1H - 2)) { rr = 1 + (v >> 1); cc = (v & 1) ? S1W - 1 : 0; return true; }
    return false;
  };
  v2<T> fr[S1NR], fh[S1NH];
#pragma unroll
  for (int q = 0; q < S1NR; ++q) {         // issue every tile load first
    int rr, cc;
    const bool in = rpos(q, rr, cc);
    const int k = r0 + rr, j = c0 + cc;
    fr[q] = (in && j > 0 && j < n && k > 0 && k < n) ? f[(size_t)k * p + j] : mk<T>(0, 0);
  }
#pragma unroll
  for (int q = 0; q < S1NH; ++q) {
    int rr, cc;
    const bool in = hpos(q, rr, cc);
    const int k = r0 + rr, j = c0 + cc;
    fh[q] = (in && j > 0 && j < n && k > 0 && k < n) ? f[(size_t)k * p + j] : mk<T>(0, 0);
  }
  stage_tabs(tb, L, c0, r0, tid);
  __syncthreads();
  // u' = omega f / d on the whole tile (d of the residual region kept)
  auto put_u = [&](int rr, int cc, v2<T>& fv, v2<T>& d) {
    const int k = r0 + rr, j = c0 + cc;
    v2<T> uv = mk<T>(0, 0);
    d = mk<T>(1, 0);
    if (j > 0 && j < n && k > 0 && k < n) {
      fv = cscale(fv, sc);
      d = tab_diag(tb, L, rr, cc, k, j);
      uv = cscale(cdiv(fv, d), omega);
    }
    up[rr][cc] = uv;
  };
  v2<T> dr[S1NR];
#pragma unroll
  for (int q = 0; q < S1NR; ++q) {
    int rr, cc;
    dr[q] = mk<T>(1, 0);
    if (rpos(q, rr, cc)) put_u(rr, cc, fr[q], dr[q]);
  }
#pragma unroll
  for (int q = 0; q < S1NH; ++q) {
    int rr, cc;
    v2<T> dh;
    if (hpos(q, rr, cc)) put_u(rr, cc, fh[q], dh);
  }
  __syncthreads();
  // residual r = f - A u' on the residual region (f from registers); it
  // replaces u' in the tile once every thread has read its neighbours
#pragma unroll
  for (int q = 0; q < S1NR; ++q) {
    int rr, cc;
    const bool in = rpos(q, rr, cc);
    const int k = r0 + rr, j = c0 + cc;
    v2<T> r = mk<T>(0, 0);
    if (in && j > 0 && j < n && k > 0 && k < n) r = csub(fr[q], tab_apply_d(tb, dr[q], up, rr, cc));
    fr[q] = r;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < S1NR; ++q) {
    int rr, cc;
    if (rpos(q, rr, cc)) up[rr][cc] = fr[q];
  }
  __syncthreads();
  const int J = J0 + threadIdx.x % S1CX, K = K0 + (tid / S1CX);
  if (tid < S1CX * S1CY && J < nc && K < nc) {
    const int cr = 2 * (K - K0) + 2, ccn = 2 * (J - J0) + 2;   // centre in the tile
    v2<T> acc = mk<T>(0, 0);
#pragma unroll
    for (int a = -1; a <= 1; ++a)
#pragma unroll
      for (int b = -1; b <= 1; ++b) {
        const T w = T((a == 0 ? 2 : 1) * (b == 0 ? 2 : 1));
        v2<T> r = up[cr + a][ccn + b];
        acc = mk<T>(acc.x + w * r.x, acc.y + w * r.y);
      }
    fc[(size_t)K * pitch_c + J] = cscale(acc, T(1.0 / 16.0));
  }
}

// S2 tile: 64 x TY fine nodes per block (TY = 16 on the finest levels, 4
// where the large tiles would give fewer than two blocks per CU)
template <int TY_> struct S2Tile {
  static constexpr int TX = 64, TY = TY_;
  static constexpr int W = TX + 2, H = TY + 2;
  static constexpr int CW = W / 2 + 2, CH = H / 2 + 2;            // coarse correction tile
  static constexpr int NH = (H * W - TX * TY + 255) / 256;       // halo points per thread
};
using S2Big = S2Tile<16>;
using S2Small = S2Tile<4>;

// S2: the thread's output points (column 1 + tx, rows 1 + ty + 4q) keep f in
// registers; only w = u' + P e_c needs an LDS tile.
template <typename T, typename TL>
__global__ void __launch_bounds__(256) k_s2_zero(Level<T> L, const v2<T>* __restrict__ f,
                                                 const double* __restrict__ fs, T omega,
                                                 const v2<T>* __restrict__ ec, int pitch_c,
                                                 v2<T>* __restrict__ u) {
  constexpr int S2TX = TL::TX, S2TY = TL::TY, S2W = TL::W, S2H = TL::H, S2CW = TL::CW, S2CH = TL::CH;
  constexpr int S2NH = TL::NH;
  __shared__ v2<T> wl[S2H][S2W];
  __shared__ v2<T> el[S2CH][S2CW];
  __shared__ TileTabs<T, S2W, S2H> tb;
  const int n = L.n, p = L.pitch, nc = n / 2;
  const int tid = threadIdx.x + 64 * threadIdx.y;
  const int j0 = 1 + blockIdx.x * S2TX - 1, k0 = 1 + blockIdx.y * S2TY - 1;   // tile origin (halo)
  const int J0 = j0 >> 1, K0 = k0 >> 1;                                       // coarse origin
  const T sc = fs ? (T)*fs : T(1);
  constexpr int NLC = (S2CH * S2CW + 255) / 256;
  constexpr int NO = S2TY / 4;                                                // output rows per thread
  auto hpos = [&](int q, int& rr, int& cc) {
    const int h = tid + 256 * q;                 // halo: rows 0 and S2H-1, columns 0 and S2W-1
    if (h < S2W) { rr = 0; cc = h; return true; }
    if (h < 2 * S2W) { rr = S2H - 1; cc = h - S2W; return true; }
    const int v = h - 2 * S2W;
    if (v < 2 * (S2H - 2)) { rr = 1 + (v >> 1); cc = (v & 1) ? S2W - 1 : 0; return true; }
    return false;
  };
  const int occ = 1 + threadIdx.x;
  v2<T> fo[NO], fh[S2NH], er[NLC];
#pragma unroll
  for (int q = 0; q < NO; ++q) {           // issue every tile load first
    const int k = k0 + 1 + threadIdx.y + 4 * q, j = j0 + occ;
    fo[q] = (j > 0 && j < n && k > 0 && k < n) ? f[(size_t)k * p + j] : mk<T>(0, 0);
  }
#pragma unroll
  for (int q = 0; q < S2NH; ++q) {
    int rr, cc;
    const bool in = hpos(q, rr, cc);
    const int k = k0 + rr, j = j0 + cc;
    fh[q] = (in && j > 0 && j < n && k > 0 && k < n) ? f[(size_t)k * p + j] : mk<T>(0, 0);
  }
#pragma unroll
  for (int q = 0; q < NLC; ++q) {
    const int idx = tid + 256 * q;
    const int K = K0 + idx / S2CW, J = J0 + idx % S2CW;
    er[q] = (idx < S2CH * S2CW && J > 0 && J < nc && K > 0 && K < nc) ? ec[(size_t)K * pitch_c + J]
                                                                      : mk<T>(0, 0);
  }
  stage_tabs(tb, L, j0, k0, tid);
#pragma unroll
  for (int q = 0; q < NLC; ++q) {
    const int idx = tid + 256 * q;
    if (idx < S2CH * S2CW) el[idx / S2CW][idx % S2CW] = er[q];
  }
  __syncthreads();
  // w = omega f / d + P e_c (bilinear: mean of the up to four coarse
  // neighbours); d and 1/|d|^2 of the output nodes are kept for the sweep
  auto put_w = [&](int rr, int cc, v2<T>& fv, v2<T>& d, T& inv) {
    const int k = k0 + rr, j = j0 + cc;
    v2<T> wv = mk<T>(0, 0);
    d = mk<T>(1, 0);
    inv = T(1);
    if (j > 0 && j < n && k > 0 && k < n) {
      fv = cscale(fv, sc);
      const int Ja = (j >> 1) - J0, Jb = ((j + 1) >> 1) - J0, Ka = (k >> 1) - K0, Kb = ((k + 1) >> 1) - K0;
      const v2<T> s = cadd(cadd(el[Ka][Ja], el[Ka][Jb]), cadd(el[Kb][Ja], el[Kb][Jb]));
      d = tab_diag(tb, L, rr, cc, k, j);
      inv = recipT(cabs2(d));
      wv = cadd(cscale(cdiv_inv(fv, d, inv), omega), cscale(s, T(0.25)));
    }
    wl[rr][cc] = wv;
  };
  v2<T> dq[NO];
  T iq[NO];
#pragma unroll
  for (int q = 0; q < NO; ++q) put_w(1 + threadIdx.y + 4 * q, occ, fo[q], dq[q], iq[q]);
#pragma unroll
  for (int q = 0; q < S2NH; ++q) {
    int rr, cc;
    v2<T> dh;
    T ih;
    if (hpos(q, rr, cc)) put_w(rr, cc, fh[q], dh, ih);
  }
  __syncthreads();
  const int j = j0 + occ;
  if (j >= n) return;
#pragma unroll
  for (int q = 0; q < NO; ++q) {
    const int rr = 1 + threadIdx.y + 4 * q;
    const int k = k0 + rr;
    if (k >= n) break;
    const v2<T> res = csub(fo[q], tab_apply_d(tb, dq[q], wl, rr, occ));
    u[(size_t)k * p + j] = cadd(wl[rr][occ], cscale(cdiv_inv(res, dq[q], iq[q]), omega));
  }
}

// S1 on two consecutive levels in one launch: level l on the 25 x 73 nodes
// whose residual restricts to the 11 x 35 tile of level l+1 that the second
// pass needs, then level l+1 on that tile, restricted to 4 x 16 points of
// level l+2.  Blocks overlap on level l and compute the same values there.
// Each block stores its own 8 x 32 part of f on level l+1 (read later by the
// post-smoothing) and its 4 x 16 points of f on level l+2.
template <typename T>
__global__ void __launch_bounds__(1024) k_s1_pair(Level<T> Lf, Level<T> Lc, const v2<T>* __restrict__ f,
                                                 const double* __restrict__ fs, T omega,
                                                 v2<T>* __restrict__ f1, int pitch1, v2<T>* __restrict__ f2,
                                                 int pitch2) {
  using TC = S1Small;                                   // level l+1 tile: 11 x 35, outputs 4 x 16
  constexpr int CW = TC::W, CH = TC::H, CRW = TC::RW, CRH = TC::RH;
  constexpr int FW = 2 * CW + 3, FH = 2 * CH + 3;       // level l tile: 25 x 73
  constexpr int RW = FW - 2, RH = FH - 2;               // its residual region: 23 x 71
  constexpr int NT = 1024;                              // threads (64 x 16)
  constexpr int NR = (RH * RW + NT - 1) / NT, NH = (FH * FW - RH * RW + NT - 1) / NT;
  constexpr int NC = (CH * CW + NT - 1) / NT, NCR = (CRH * CRW + NT - 1) / NT;
  static_assert(NH == 1 && TC::NH == 1, "one halo node per thread");
  __shared__ v2<T> up0[FH][FW];                         // u', then r on level l
  __shared__ v2<T> ft1[CH][CW];                         // f on level l+1
  __shared__ v2<T> up1[CH][CW];                         // u', then r on level l+1
  __shared__ TileTabs<T, FW, FH> tb0;
  __shared__ TileTabs<T, CW, CH> tb1;
  const int n = Lf.n, p = Lf.pitch, n1 = Lc.n, n2 = n1 / 2;
  const int tid = threadIdx.x + 64 * threadIdx.y;
  const int J2 = 1 + blockIdx.x * TC::CX, K2 = 1 + blockIdx.y * TC::CY;   // level l+2 origin
  const int c1 = 2 * J2 - 2, r1 = 2 * K2 - 2;                             // level l+1 tile origin
  const int c0 = 2 * c1 - 2, r0 = 2 * r1 - 2;                             // level l tile origin
  auto rpos = [&](int q, int& rr, int& cc) {
    const int idx = tid + NT * q;
    rr = 1 + idx / RW;
    cc = 1 + idx % RW;
    return idx < RH * RW;
  };
  auto hpos = [&](int& rr, int& cc) {
    const int h = tid;
    if (h < FW) { rr = 0; cc = h; return true; }
    if (h < 2 * FW) { rr = FH - 1; cc = h - FW; return true; }
    const int v = h - 2 * FW;
    if (v < 2 * (FH - 2)) { rr = 1 + (v >> 1); cc = (v & 1) ? FW - 1 : 0; return true; }
    return false;
  };
  auto interior = [](int k, int j, int m) { return j > 0 && j < m && k > 0 && k < m; };
  // every load first
  v2<T> fr[NR], fh;
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    int rr, cc;
    const bool in = rpos(q, rr, cc);
    const int k = r0 + rr, j = c0 + cc;
    fr[q] = (in && interior(k, j, n)) ? f[(size_t)k * p + j] : mk<T>(0, 0);
  }
  {
    int rr, cc;
    const bool in = hpos(rr, cc);
    const int k = r0 + rr, j = c0 + cc;
    fh = (in && interior(k, j, n)) ? f[(size_t)k * p + j] : mk<T>(0, 0);
  }
  if (tid < FW + FH) stage_tabs(tb0, Lf, c0, r0, tid);
  if (tid >= 128 && tid < 128 + CW + CH) stage_tabs(tb1, Lc, c1, r1, tid - 128);
  const T sc = fs ? (T)*fs : T(1);
  __syncthreads();
  // level l: u' = omega f / d on the tile
  auto put_u = [&](int rr, int cc, v2<T>& fv) {
    const int k = r0 + rr, j = c0 + cc;
    v2<T> uv = mk<T>(0, 0);
    if (interior(k, j, n)) {
      fv = cscale(fv, sc);
      uv = cscale(cdiv(fv, tab_diag(tb0, Lf, rr, cc, k, j)), omega);
    }
    up0[rr][cc] = uv;
  };
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    int rr, cc;
    if (rpos(q, rr, cc)) put_u(rr, cc, fr[q]);
  }
  {
    int rr, cc;
    if (hpos(rr, cc)) put_u(rr, cc, fh);
  }
  __syncthreads();
  // level l: r = f - A u' on the residual region, then in place of u'
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    int rr, cc;
    const bool in = rpos(q, rr, cc);
    const int k = r0 + rr, j = c0 + cc;
    v2<T> r = mk<T>(0, 0);
    if (in && interior(k, j, n)) r = csub(fr[q], tab_apply(tb0, Lf, up0, rr, cc, k, j));
    fr[q] = r;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    int rr, cc;
    if (rpos(q, rr, cc)) up0[rr][cc] = fr[q];
  }
  __syncthreads();
  // level l+1: f by full weighting on the 11 x 35 tile (zero off the interior);
  // the block's own 8 x 32 part goes to memory
  auto fw = [&](v2<T> (*w)[FW], int cr, int cn) {
    v2<T> acc = mk<T>(0, 0);
#pragma unroll
    for (int a = -1; a <= 1; ++a)
#pragma unroll
      for (int b = -1; b <= 1; ++b) {
        const T wt = T((a == 0 ? 2 : 1) * (b == 0 ? 2 : 1));
        const v2<T> r = w[cr + a][cn + b];
        acc = mk<T>(acc.x + wt * r.x, acc.y + wt * r.y);
      }
    return cscale(acc, T(1.0 / 16.0));
  };
  v2<T> f1r[NC];
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    const int idx = tid + NT * q, rr = idx / CW, cc = idx % CW, K = r1 + rr, J = c1 + cc;
    v2<T> v = mk<T>(0, 0);
    if (idx < CH * CW && interior(K, J, n1)) {
      v = fw(up0, 2 * rr + 2, 2 * cc + 2);           // level-l node 2K, 2J at tile position 2rr+2, 2cc+2
      // own part: rows 1..8, columns 1..32 of the tile (the last block row /
      // column also takes the rest of the interior)
      const bool own_r = rr >= 1 && (rr <= 2 * TC::CY || blockIdx.y + 1 == gridDim.y);
      const bool own_c = cc >= 1 && (cc <= 2 * TC::CX || blockIdx.x + 1 == gridDim.x);
      if (own_r && own_c) f1[(size_t)K * pitch1 + J] = v;
    }
    f1r[q] = v;
    if (idx < CH * CW) ft1[rr][cc] = v;
  }
  __syncthreads();
  // level l+1: u' on the tile, r on its residual region, full weighting
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    const int idx = tid + NT * q, rr = idx / CW, cc = idx % CW, K = r1 + rr, J = c1 + cc;
    if (idx < CH * CW)
      up1[rr][cc] = interior(K, J, n1) ? cscale(cdiv(f1r[q], tab_diag(tb1, Lc, rr, cc, K, J)), omega)
                                       : mk<T>(0, 0);
  }
  __syncthreads();
  v2<T> r1v[NCR];
#pragma unroll
  for (int q = 0; q < NCR; ++q) {
    const int idx = tid + NT * q, rr = 1 + idx / CRW, cc = 1 + idx % CRW, K = r1 + rr, J = c1 + cc;
    v2<T> r = mk<T>(0, 0);
    if (idx < CRH * CRW && interior(K, J, n1)) r = csub(ft1[rr][cc], tab_apply(tb1, Lc, up1, rr, cc, K, J));
    r1v[q] = r;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NCR; ++q) {
    const int idx = tid + NT * q;
    if (idx < CRH * CRW) up1[1 + idx / CRW][1 + idx % CRW] = r1v[q];
  }
  __syncthreads();
  const int J = J2 + tid % TC::CX, K = K2 + tid / TC::CX;
  if (tid < TC::CX * TC::CY && J < n2 && K < n2) {
    const int cr = 2 * (K - K2) + 2, cn = 2 * (J - J2) + 2;
    v2<T> acc = mk<T>(0, 0);
#pragma unroll
    for (int a = -1; a <= 1; ++a)
#pragma unroll
      for (int b = -1; b <= 1; ++b) {
        const T wt = T((a == 0 ? 2 : 1) * (b == 0 ? 2 : 1));
        const v2<T> r = up1[cr + a][cn + b];
        acc = mk<T>(acc.x + wt * r.x, acc.y + wt * r.y);
      }
    f2[(size_t)K * pitch2 + J] = cscale(acc, T(1.0 / 16.0));
  }
}

// S2 on two consecutive levels in one launch: level l+1 on the region that
// the prolongation of a 64 x 4 tile of level l reads (5 x 35 nodes, from w on
// 7 x 37 nodes), then level l on the tile.  Blocks overlap on level l+1 and
// compute the same values there; u of level l+1 stays on chip.
//   ff, fs: f of level l (fs: optional device scale);  fc: f of level l+1;
//   ecc: e of level l+2 (pitch_cc);  u: output of level l.
template <typename T>
__global__ void __launch_bounds__(256) k_s2_pair(Level<T> Lf, Level<T> Lc, const v2<T>* __restrict__ ff,
                                                 const double* __restrict__ fs, const v2<T>* __restrict__ fc,
                                                 const v2<T>* __restrict__ ecc, int pitch_cc, T omega,
                                                 v2<T>* __restrict__ u) {
  using TL = S2Small;
  constexpr int FW = TL::W, FH = TL::H;                 // fine w tile (66 x 6)
  constexpr int EW = TL::CW, EH = TL::CH;               // e of level l+1 (35 x 5)
  constexpr int CW = EW + 2, CH = EH + 2;               // w of level l+1 (37 x 7)
  constexpr int QW = 20, QH = 5;                        // e of level l+2 under it
  constexpr int NCW = (CW * CH + 255) / 256;
  static_assert(TL::TY == 4 && TL::NH == 1 && QW * QH <= 256, "tile layout");
  __shared__ v2<T> wf[FH][FW];
  __shared__ v2<T> e1[EH][EW];
  __shared__ v2<T> w1[CH][CW];
  __shared__ v2<T> e2[QH][QW];
  __shared__ TileTabs<T, FW, FH> tbf;
  __shared__ TileTabs<T, CW, CH> tbc;
  const int n = Lf.n, p = Lf.pitch, nc = Lc.n, pc = Lc.pitch, ncc = nc / 2;
  const int tid = threadIdx.x + 64 * threadIdx.y;
  const int j0 = blockIdx.x * TL::TX, k0 = blockIdx.y * TL::TY;    // fine tile origin (halo)
  const int J0 = j0 >> 1, K0 = k0 >> 1;                            // e1 origin
  const int Q0 = (J0 >> 1) - 1, R0 = (K0 >> 1) - 1;                // e2 origin (J0, K0 even)
  auto hpos = [&](int& rr, int& cc) {
    const int h = tid;                            // fine halo: rows 0 and FH-1, columns 0 and FW-1
    if (h < FW) { rr = 0; cc = h; return true; }
    if (h < 2 * FW) { rr = FH - 1; cc = h - FW; return true; }
    const int v = h - 2 * FW;
    if (v < 2 * (FH - 2)) { rr = 1 + (v >> 1); cc = (v & 1) ? FW - 1 : 0; return true; }
    return false;
  };
  // every load first: f of level l (output node + one halo node), f of level
  // l+1 on the w1 region, e of level l+2, the tables of both levels
  const int orr = 1 + threadIdx.y, occ = 1 + threadIdx.x;
  v2<T> fo, fh, fcv[NCW], eq = mk<T>(0, 0);
  {
    const int k = k0 + orr, j = j0 + occ;
    fo = (j > 0 && j < n && k > 0 && k < n) ? ff[(size_t)k * p + j] : mk<T>(0, 0);
    int rr, cc;
    const bool in = hpos(rr, cc);
    const int kh = k0 + rr, jh = j0 + cc;
    fh = (in && jh > 0 && jh < n && kh > 0 && kh < n) ? ff[(size_t)kh * p + jh] : mk<T>(0, 0);
  }
#pragma unroll
  for (int q = 0; q < NCW; ++q) {
    const int idx = tid + 256 * q, K = K0 - 1 + idx / CW, J = J0 - 1 + idx % CW;
    fcv[q] = (idx < CW * CH && J > 0 && J < nc && K > 0 && K < nc) ? fc[(size_t)K * pc + J] : mk<T>(0, 0);
  }
  if (tid < QW * QH) {
    const int K = R0 + tid / QW, J = Q0 + tid % QW;
    if (J > 0 && J < ncc && K > 0 && K < ncc) eq = ecc[(size_t)K * pitch_cc + J];
  }
  if (tid < CW + CH) stage_tabs(tbc, Lc, J0 - 1, K0 - 1, tid);
  if (tid >= 64 && tid < 64 + FW + FH) stage_tabs(tbf, Lf, j0, k0, tid - 64);
  if (tid < QW * QH) e2[tid / QW][tid % QW] = eq;
  __syncthreads();
  // level l+1: w = omega f / d + P e2 on 7 x 37 nodes (d, 1/|d|^2 kept)
  v2<T> dc[NCW];
  T ic[NCW];
#pragma unroll
  for (int q = 0; q < NCW; ++q) {
    const int idx = tid + 256 * q;
    dc[q] = mk<T>(1, 0);
    ic[q] = T(1);
    if (idx < CW * CH) {
      const int rr = idx / CW, cc = idx % CW, K = K0 - 1 + rr, J = J0 - 1 + cc;
      v2<T> wv = mk<T>(0, 0);
      if (J > 0 && J < nc && K > 0 && K < nc) {
        const int Ja = (J >> 1) - Q0, Jb = ((J + 1) >> 1) - Q0, Ka = (K >> 1) - R0, Kb = ((K + 1) >> 1) - R0;
        const v2<T> s = cadd(cadd(e2[Ka][Ja], e2[Ka][Jb]), cadd(e2[Kb][Ja], e2[Kb][Jb]));
        dc[q] = tab_diag(tbc, Lc, rr, cc, K, J);
        ic[q] = recipT(cabs2(dc[q]));
        wv = cadd(cscale(cdiv_inv(fcv[q], dc[q], ic[q]), omega), cscale(s, T(0.25)));
      }
      w1[rr][cc] = wv;
    }
  }
  __syncthreads();
  // level l+1: u = w + omega (f - A w) / d on the inner 5 x 35 nodes
#pragma unroll
  for (int q = 0; q < NCW; ++q) {
    const int idx = tid + 256 * q;
    const int rr = idx / CW, cc = idx % CW;
    if (idx < CW * CH && rr >= 1 && rr <= EH && cc >= 1 && cc <= EW) {
      const int K = K0 - 1 + rr, J = J0 - 1 + cc;
      v2<T> o = mk<T>(0, 0);
      if (J > 0 && J < nc && K > 0 && K < nc) {
        const v2<T> res = csub(fcv[q], tab_apply_d(tbc, dc[q], w1, rr, cc));
        o = cadd(w1[rr][cc], cscale(cdiv_inv(res, dc[q], ic[q]), omega));
      }
      e1[rr - 1][cc - 1] = o;
    }
  }
  __syncthreads();
  // level l: w = omega f / d + P e1 on the 6 x 66 tile
  const T sc = fs ? (T)*fs : T(1);
  auto put_w = [&](int rr, int cc, v2<T>& fv, v2<T>& d, T& inv) {
    const int k = k0 + rr, j = j0 + cc;
    v2<T> wv = mk<T>(0, 0);
    d = mk<T>(1, 0);
    inv = T(1);
    if (j > 0 && j < n && k > 0 && k < n) {
      fv = cscale(fv, sc);
      const int Ja = (j >> 1) - J0, Jb = ((j + 1) >> 1) - J0, Ka = (k >> 1) - K0, Kb = ((k + 1) >> 1) - K0;
      const v2<T> s = cadd(cadd(e1[Ka][Ja], e1[Ka][Jb]), cadd(e1[Kb][Ja], e1[Kb][Jb]));
      d = tab_diag(tbf, Lf, rr, cc, k, j);
      inv = recipT(cabs2(d));
      wv = cadd(cscale(cdiv_inv(fv, d, inv), omega), cscale(s, T(0.25)));
    }
    wf[rr][cc] = wv;
  };
  v2<T> dq;
  T iq;
  put_w(orr, occ, fo, dq, iq);
  {
    int rr, cc;
    v2<T> dh;
    T ih;
    if (hpos(rr, cc)) put_w(rr, cc, fh, dh, ih);
  }
  __syncthreads();
  const int k = k0 + orr, j = j0 + occ;
  if (j >= n || k >= n) return;
  const v2<T> res = csub(fo, tab_apply_d(tbf, dq, wf, orr, occ));
  u[(size_t)k * p + j] = cadd(wf[orr][occ], cscale(cdiv_inv(res, dq, iq), omega));
}

// ----------------------------------------------------------------------------
// Coarse tail of the zero-guess V-cycle: the levels with n <= TN are held
// whole in LDS (one node row of halo on each side is the zero boundary).
//   k_tail_down: the S1 passes of every tail level, then u_c = Ainv f_c on the
//     coarsest level.  Each block repeats the (small) S1 passes and takes 16
//     rows of Ainv, so the coarsest solve needs no second launch; block 0
//     stores the restricted right-hand sides the up pass needs.
//   k_tail_up: the S2 passes from the coarsest level up; each block repeats
//     the passes below the top tail level and takes 16 rows of the top one.
// The arithmetic per node is that of k_s1_zero / k_s2_zero / k_coarse_solve.
constexpr int TN = 64, TBW = TN + 1, TSW = TN / 2 + 1;
constexpr int TT = 1024;                       // threads per tail block
constexpr int TROWS = TT / 64;                 // Ainv rows per tail-down block
template <int LV> constexpr int tail_np() {    // nodes per thread on tail level LV
  return (((TN >> LV) + 1) * ((TN >> LV) + 1) + TT - 1) / TT;
}

// nodes (k, j) of a level of size n (0..n both ways) owned by thread t
__device__ __forceinline__ bool tail_node(int t, int q, int n, int& k, int& j) {
  const int i = t + TT * q, w = n + 1;
  k = i / w;
  j = i - k * w;
  return i < w * w;
}

template <typename T, int LV, int NP>
__device__ __forceinline__ void tail_load(v2<T> (&fr)[NP], const TailArgs<T>& A, int t) {
  const int n = A.L[LV].n, p = A.pitch[LV];
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    int k, j;
    const bool in = tail_node(t, q, n, k, j);
    fr[q] = (in && j > 0 && j < n && k > 0 && k < n) ? A.f[LV][(size_t)k * p + j] : mk<T>(0, 0);
  }
}

// Tables of every tail level, staged once at kernel start (130 threads per
// level); the caller's barrier publishes them.
template <typename T>
__device__ __forceinline__ void tail_tabs(TileTabs<T, TBW, TBW> (&tb)[TMAXL], const TailArgs<T>& A, int t) {
  const int lv = t / (2 * TBW);
  if (lv < TMAXL && lv < A.nl) stage_tabs(tb[lv], A.L[lv], 0, 0, t - lv * 2 * TBW);
}

// one S1 pass on tail level LV: f (registers, scaled by sc) -> f of LV + 1 in
// sml (and in global memory when store).  Entered after a barrier.
template <typename T, int LV, int NP>
__device__ __forceinline__ void tail_s1(const TailArgs<T>& A, v2<T> (&fr)[NP], T sc, v2<T> (*big)[TBW],
                                        v2<T> (*sml)[TSW], const TileTabs<T, TBW, TBW>& tb, int t,
                                        bool store) {
  const Level<T>& L = A.L[LV];
  const int n = L.n, nc = n / 2;
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    int k, j;
    if (!tail_node(t, q, n, k, j)) break;
    v2<T> uv = mk<T>(0, 0);
    if (j > 0 && j < n && k > 0 && k < n) {
      fr[q] = cscale(fr[q], sc);
      uv = cscale(cdiv(fr[q], tab_diag(tb, L, k, j, k, j)), A.omega);
    }
    big[k][j] = uv;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    int k, j;
    const bool in = tail_node(t, q, n, k, j);
    v2<T> r = mk<T>(0, 0);
    if (in && j > 0 && j < n && k > 0 && k < n) r = csub(fr[q], tab_apply(tb, L, big, k, j, k, j));
    fr[q] = r;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    int k, j;
    if (tail_node(t, q, n, k, j)) big[k][j] = fr[q];
  }
  __syncthreads();
  const int pc = A.pitch[LV + 1];
  for (int i = t; i < (nc + 1) * (nc + 1); i += TT) {
    const int K = i / (nc + 1), J = i - K * (nc + 1);
    v2<T> acc = mk<T>(0, 0);
    if (J > 0 && J < nc && K > 0 && K < nc) {
#pragma unroll
      for (int a = -1; a <= 1; ++a)
#pragma unroll
        for (int b = -1; b <= 1; ++b) {
          const T w = T((a == 0 ? 2 : 1) * (b == 0 ? 2 : 1));
          const v2<T> r = big[2 * K + a][2 * J + b];
          acc = mk<T>(acc.x + w * r.x, acc.y + w * r.y);
        }
      acc = cscale(acc, T(1.0 / 16.0));
      if (store) A.f[LV + 1][(size_t)K * pc + J] = acc;
    }
    sml[K][J] = acc;
  }
  __syncthreads();
}

// S1 passes of levels LV .. nl-1 (f of level LV already in registers)
template <typename T, int LV>
__device__ __forceinline__ void tail_down_from(const TailArgs<T>& A, v2<T> (&fr)[tail_np<LV>()], T sc,
                                               v2<T> (*big)[TBW], v2<T> (*sml)[TSW],
                                               const TileTabs<T, TBW, TBW> (&tb)[TMAXL], int t, bool store) {
  tail_s1<T, LV>(A, fr, sc, big, sml, tb[LV], t, store);
  if constexpr (LV + 1 < TMAXL) {
    if (LV + 1 < A.nl) {
      constexpr int NQ = tail_np<LV + 1>();
      v2<T> fn[NQ];
      const int n = A.L[LV + 1].n;
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        int k, j;
        fn[q] = tail_node(t, q, n, k, j) ? sml[k][j] : mk<T>(0, 0);
      }
      tail_down_from<T, LV + 1>(A, fn, T(1), big, sml, tb, t, store);
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(TT) k_tail_down(TailArgs<T> A) {
  __shared__ v2<T> big[TBW][TBW];
  __shared__ v2<T> sml[TSW][TSW];
  __shared__ TileTabs<T, TBW, TBW> tb[TMAXL];
  const int t = threadIdx.x;
  const int m = A.nc - 1, N = m * m;
  const int row = blockIdx.x * TROWS + (t >> 6), lane = t & 63;
  // this wave's row of Ainv (first 256 columns) is fetched while the S1 passes run
  constexpr int NA = 4;
  double2 ar[NA];
#pragma unroll
  for (int i = 0; i < NA; ++i) {
    const int c = lane + 64 * i;
    ar[i] = (row < N && c < N) ? A.Ainv[(size_t)row * N + c] : make_double2(0, 0);
  }
  v2<T> fr[tail_np<0>()];
  tail_load<T, 0>(fr, A, t);
  tail_tabs(tb, A, t);
  const T sc = A.fs ? (T)*A.fs : T(1);
  __syncthreads();
  tail_down_from<T, 0>(A, fr, sc, big, sml, tb, t, blockIdx.x == 0);
  if (row >= N) return;
  double sr = 0, si = 0;
#pragma unroll
  for (int i = 0; i < NA; ++i) {
    const int c = lane + 64 * i;
    if (c < N) {
      const v2<double> fv = cvt<double>(sml[c / m + 1][c % m + 1]);
      sr += ar[i].x * fv.x - ar[i].y * fv.y;
      si += ar[i].x * fv.y + ar[i].y * fv.x;
    }
  }
  for (int c = lane + 64 * NA; c < N; c += 64) {
    const double2 av = A.Ainv[(size_t)row * N + c];
    const v2<double> fv = cvt<double>(sml[c / m + 1][c % m + 1]);
    sr += av.x * fv.x - av.y * fv.y;
    si += av.x * fv.y + av.y * fv.x;
  }
  sr = wave_sum(sr);
  si = wave_sum(si);
  if (lane == 0) {
    const int k = row / m + 1, j = row % m + 1;
    A.u[A.nl][(size_t)k * A.pitch[A.nl] + j] = mk<T>((T)sr, (T)si);
  }
}

// one S2 pass on tail level LV >= 1: e of level LV + 1 in sml -> e of level
// LV in sml.  Entered after a barrier.
template <typename T, int LV, int NP>
__device__ __forceinline__ void tail_s2(const TailArgs<T>& A, v2<T> (&fr)[NP], T sc, v2<T> (*big)[TBW],
                                        v2<T> (*sml)[TSW], const TileTabs<T, TBW, TBW>& tb, int t) {
  const Level<T>& L = A.L[LV];
  const int n = L.n;
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    int k, j;
    if (!tail_node(t, q, n, k, j)) break;
    v2<T> wv = mk<T>(0, 0);
    if (j > 0 && j < n && k > 0 && k < n) {
      fr[q] = cscale(fr[q], sc);
      const int Ja = j >> 1, Jb = (j + 1) >> 1, Ka = k >> 1, Kb = (k + 1) >> 1;
      const v2<T> s = cadd(cadd(sml[Ka][Ja], sml[Ka][Jb]), cadd(sml[Kb][Ja], sml[Kb][Jb]));
      wv = cadd(cscale(cdiv(fr[q], tab_diag(tb, L, k, j, k, j)), A.omega), cscale(s, T(0.25)));
    }
    big[k][j] = wv;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    int k, j;
    const bool in = tail_node(t, q, n, k, j);
    v2<T> o = mk<T>(0, 0);
    if (in && j > 0 && j < n && k > 0 && k < n) {
      const v2<T> d = tab_diag(tb, L, k, j, k, j);
      const v2<T> res = csub(fr[q], tab_apply(tb, L, big, k, j, k, j));
      o = cadd(big[k][j], cscale(cdiv(res, d), A.omega));
    }
    fr[q] = o;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    int k, j;
    if (tail_node(t, q, n, k, j)) sml[k][j] = fr[q];
  }
  __syncthreads();
}

// The top tail level's S2 pass on output rows [ka, kb) only (w on rows
// ka-1 .. kb); nodes row-major from row ka-1.
constexpr int TUPR = 16;                                        // output rows per up block
constexpr int TNP_TOP = ((TUPR + 2) * TBW + TT - 1) / TT;
__device__ __forceinline__ bool tail_row_node(int t, int q, int n, int ka, int kb, int& k, int& j) {
  const int i = t + TT * q, w = n + 1;
  const int r = i / w;
  k = ka - 1 + r;
  j = i - r * w;
  return k <= kb;
}
template <typename T>
__device__ __forceinline__ void tail_s2_rows(const TailArgs<T>& A, v2<T> (&fr)[TNP_TOP], T sc,
                                             v2<T> (*big)[TBW], v2<T> (*sml)[TSW],
                                             const TileTabs<T, TBW, TBW>& tb, int t, int ka, int kb) {
  const Level<T>& L = A.L[0];
  const int n = L.n;
#pragma unroll
  for (int q = 0; q < TNP_TOP; ++q) {
    int k, j;
    if (!tail_row_node(t, q, n, ka, kb, k, j)) break;
    v2<T> wv = mk<T>(0, 0);
    if (j > 0 && j < n && k > 0 && k < n) {
      fr[q] = cscale(fr[q], sc);
      const int Ja = j >> 1, Jb = (j + 1) >> 1, Ka = k >> 1, Kb = (k + 1) >> 1;
      const v2<T> s = cadd(cadd(sml[Ka][Ja], sml[Ka][Jb]), cadd(sml[Kb][Ja], sml[Kb][Jb]));
      wv = cadd(cscale(cdiv(fr[q], tab_diag(tb, L, k, j, k, j)), A.omega), cscale(s, T(0.25)));
    }
    big[k][j] = wv;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < TNP_TOP; ++q) {
    int k, j;
    if (!tail_row_node(t, q, n, ka, kb, k, j)) break;
    if (k >= ka && k < kb && j > 0 && j < n) {
      const v2<T> d = tab_diag(tb, L, k, j, k, j);
      const v2<T> res = csub(fr[q], tab_apply(tb, L, big, k, j, k, j));
      A.u[0][(size_t)k * A.pitch[0] + j] = cadd(big[k][j], cscale(cdiv(res, d), A.omega));
    }
  }
}

// Up pass: block b repeats the S2 passes below the top tail level and takes
// rows [1 + 16 b, 17 + 16 b) of the top level.
template <typename T>
__global__ void __launch_bounds__(TT) k_tail_up(TailArgs<T> A) {
  static_assert(TMAXL == 4, "the up pass is written out for four tail levels");
  __shared__ v2<T> big[TBW][TBW];
  __shared__ v2<T> sml[TSW][TSW];
  __shared__ TileTabs<T, TBW, TBW> tb[TMAXL];
  const int t = threadIdx.x;
  const int n0 = A.L[0].n;
  const int ka = 1 + blockIdx.x * TUPR, kb = min(n0, ka + TUPR);
  // every load up front: e on the coarsest level, f of each tail level, tables
  {
    const int nc = A.nc, p = A.pitch[A.nl];
    for (int i = t; i < (nc + 1) * (nc + 1); i += TT) {
      const int K = i / (nc + 1), J = i - K * (nc + 1);
      sml[K][J] = (J > 0 && J < nc && K > 0 && K < nc) ? A.u[A.nl][(size_t)K * p + J] : mk<T>(0, 0);
    }
  }
  v2<T> f0[TNP_TOP], f1[tail_np<1>()], f2[tail_np<2>()], f3[tail_np<3>()];
#pragma unroll
  for (int q = 0; q < TNP_TOP; ++q) {
    int k, j;
    const bool in = tail_row_node(t, q, n0, ka, kb, k, j);
    f0[q] = (in && j > 0 && j < n0 && k > 0 && k < n0) ? A.f[0][(size_t)k * A.pitch[0] + j] : mk<T>(0, 0);
  }
  if (A.nl > 1) tail_load<T, 1>(f1, A, t);
  if (A.nl > 2) tail_load<T, 2>(f2, A, t);
  if (A.nl > 3) tail_load<T, 3>(f3, A, t);
  tail_tabs(tb, A, t);
  const T sc = A.fs ? (T)*A.fs : T(1);
  __syncthreads();
  if (A.nl > 3) tail_s2<T, 3>(A, f3, T(1), big, sml, tb[3], t);
  if (A.nl > 2) tail_s2<T, 2>(A, f2, T(1), big, sml, tb[2], t);
  if (A.nl > 1) tail_s2<T, 1>(A, f1, T(1), big, sml, tb[1], t);
  tail_s2_rows<T>(A, f0, sc, big, sml, tb[0], t, ka, kb);
}

// ----------------------------------------------------------------------------
// CCCS.  Step 1: residual r = f - A u and both channel projections on 64x64
// tiles; r is never stored.
//   rho^A[k][i] = sum_j w_j phi_i(j) r[k][j]   -> partA[tile_x][k][i]
//   rho^B[j][l] = sum_k w_k varphi_l(k) r[k][j] -> partB[tile_y][j][l]
// Thread = one column, PT / W rows; the block's W waves cover 64 rows (W = 8
// or 4 where 16 waves would not fit the registers of wide channel sets).  All
// loads are issued together at the start: u on the tile and its halo into
// LDS, f, the column and row tables.  The column sums (rho^B) accumulate in
// registers over the wave's rows; the residual tile then goes to LDS, where
// the row sums (rho^A) run with lane = row over a slice of columns per wave.
// Both are combined over the waves in a fixed order (no shuffles).
constexpr int PT = 64;
template <typename T, int MC> struct ProjCfg {
  static constexpr int W = MC * sizeof(T) >= 256 ? 4 : (MC * sizeof(T) >= 64 ? 8 : 16);   // waves
  static constexpr int R = PT / W;                           // rows per wave
};

template <typename T, int MC>
__global__ void __launch_bounds__((64 * ProjCfg<T, MC>::W)) k_cccs_project(Level<T> L, const v2<T>* __restrict__ u,
                                                          const v2<T>* __restrict__ f,
                                                          const double* __restrict__ fs, ChanTab<T> ch,
                                                          v2<T>* __restrict__ partA,
                                                          v2<T>* __restrict__ partB) {
  constexpr int PW = ProjCfg<T, MC>::W, PR = ProjCfg<T, MC>::R, NT = 64 * PW;
  constexpr int UW = PT + 2;                     // u tile with its one-node halo
  constexpr int NU = (UW * UW + NT - 1) / NT;    // u tile loads per thread
  constexpr int FR = PR < 8 ? PR : 8;            // rows of f per register batch
  constexpr int RP = PT + 1;                     // row pitch of the residual tile (odd: no bank conflicts)
  constexpr int CPW = PT / PW;                   // columns per wave in the row sums
  static_assert(PT * RP <= UW * UW, "the residual tile reuses the u tile");
  __shared__ v2<T> ut[UW][UW];
  __shared__ v2<T> rt[4][PT];                    // per tile row: py, a, c, tm
  __shared__ v2<T> wv[PT][MC];                   // w_k varphi_l(k) of the tile rows
  __shared__ v2<T> wpl[MC][PT];                  // w_j phi_i(j) of the tile columns
  __shared__ v2<T> red[64][MC + 1], redA[64][MC + 1];   // odd row pitch: lane = row without bank conflicts
  v2<T>* rtile = &ut[0][0];                      // [PT][RP] residual, after the stencil
  const int n = L.n, p = L.pitch, M = ch.M, Lc = ch.L;
  const int tx = threadIdx.x, ty = threadIdx.y, tid = tx + 64 * ty;
  const int j0 = 1 + blockIdx.x * PT, j = j0 + tx;
  const int kb = 1 + blockIdx.y * PT;
  const bool jok = j < n;
  const int jc = jok ? j : n - 1;
  const int kw = __builtin_amdgcn_readfirstlane(kb + PR * ty);   // the wave's first row
  auto clampi = [&](int x) { return x < 1 ? 1 : (x > n - 1 ? n - 1 : x); };
  // phase 1: every load at once (clamped addresses; zeros selected at the
  // LDS writes)
  v2<T> ul[NU];
#pragma unroll
  for (int q = 0; q < NU; ++q) {
    const int idx = tid + NT * q, rr = idx / UW, cc = idx - rr * UW;
    ul[q] = u[(size_t)clampi(kb - 1 + rr) * p + clampi(j0 - 1 + cc)];
  }
  v2<T> fv[FR];
#pragma unroll
  for (int q = 0; q < FR; ++q) fv[q] = f[(size_t)clampi(kw + q) * p + jc];
  const v2<T> aj = L.a[jc], cj = L.c[jc], pxj = L.px[jc], tmj = L.tm[jc];
  v2<T> tv = mk<T>(0, 0);
  if (tid < 4 * PT) {
    const int t4 = tid / PT, kc = clampi(kb + tid % PT);
    const v2<T>* tab = t4 == 0 ? L.py : (t4 == 1 ? L.a : (t4 == 2 ? L.c : L.tm));
    tv = tab[kc];
  }
  constexpr int NW = (PT * MC + NT - 1) / NT;
  v2<T> wl[NW], wq[NW];
#pragma unroll
  for (int q = 0; q < NW; ++q) {
    const int idx = tid + NT * q, l = idx % MC, c = idx / MC;
    wl[q] = ch.wvphi[(size_t)(l < Lc ? l : Lc - 1) * (n + 1) + clampi(kb + c)];
    // w_j phi_i(j): idx = i * PT + column (coalesced)
    const int i = idx / PT, cc = idx % PT;
    wq[q] = ch.wphi[(size_t)(i < M ? i : M - 1) * (n + 1) + clampi(j0 + cc)];
  }
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int q = 0; q < NU; ++q) {
    const int idx = tid + NT * q, rr = idx / UW, cc = idx - rr * UW;
    const int k = kb - 1 + rr, jj = j0 - 1 + cc;
    if (idx < UW * UW) ut[rr][cc] = (k > 0 && k < n && jj > 0 && jj < n) ? ul[q] : mk<T>(0, 0);
  }
  if (tid < 4 * PT) rt[tid / PT][tid % PT] = tv;
#pragma unroll
  for (int q = 0; q < NW; ++q) {
    const int idx = tid + NT * q;
    if (idx < PT * MC) {
      const int r = idx / MC, l = idx % MC;
      wv[r][l] = (l < Lc && kb + r < n) ? wl[q] : mk<T>(0, 0);
      const int i = idx / PT, cc = idx % PT;
      wpl[i][cc] = (i < M && j0 + cc < n) ? wq[q] : mk<T>(0, 0);
    }
  }
  const T sc = fs ? (T)*fs : T(1);
  __syncthreads();
  // phase 2: the wave's residual rows (registers) and its rho^B partials
  v2<T> accB[MC], rr_[PR];
#pragma unroll
  for (int i = 0; i < MC; ++i) accB[i] = mk<T>(0, 0);
#pragma unroll
  for (int q = 0; q < PR; ++q) rr_[q] = mk<T>(0, 0);
  const int uc = tx + 1;
#pragma unroll
  for (int q0 = 0; q0 < PR; q0 += FR) {
    if (q0 > 0) {
#pragma unroll
      for (int q = 0; q < FR; ++q) fv[q] = f[(size_t)clampi(kw + q0 + q) * p + jc];
    }
#pragma unroll
    for (int q = 0; q < FR; ++q) {
      const int k = kw + q0 + q;                        // wave-uniform row
      if (k >= n) break;
      const int rr = k - kb, ur = rr + 1;
      v2<T> r = mk<T>(0, 0);
      if (jok) {
        v2<T> d = cadd(cadd(pxj, rt[0][rr]), j > k ? tmj : rt[3][rr]);
        if (L.v12) d = cadd(d, v12_at(L, k, j));
        d.x -= L.E;
        v2<T> acc = cmul(d, ut[ur][uc]);
        acc = cfma(acc, aj, ut[ur][uc - 1]);
        acc = cfma(acc, cj, ut[ur][uc + 1]);
        acc = cfma(acc, rt[1][rr], ut[ur - 1][uc]);
        acc = cfma(acc, rt[2][rr], ut[ur + 1][uc]);
        r = csub(cscale(fv[q], sc), acc);
      }
      rr_[q0 + q] = r;
#pragma unroll
      for (int i = 0; i < MC; ++i) accB[i] = cfma(accB[i], wv[rr][i], r);
    }
  }
  __syncthreads();                               // every stencil read of u is done
#pragma unroll
  for (int q = 0; q < PR; ++q) rtile[(PR * ty + q) * RP + tx] = rr_[q];
  __syncthreads();
  // phase 3: rho^A row sums, lane = tile row, wave = a slice of CPW columns
  v2<T> accA[MC];
#pragma unroll
  for (int i = 0; i < MC; ++i) accA[i] = mk<T>(0, 0);
#pragma unroll
  for (int c = 0; c < CPW; ++c) {
    const int cc = CPW * ty + c;
    const v2<T> rv = rtile[tx * RP + cc];
#pragma unroll
    for (int i = 0; i < MC; ++i) accA[i] = cfma(accA[i], wpl[i][cc], rv);
  }
  // the waves add their sums in order (rho^B by column, rho^A by row)
  if (ty == 0)
#pragma unroll
    for (int l = 0; l < MC; ++l) {
      red[tx][l] = accB[l];
      redA[tx][l] = accA[l];
    }
  __syncthreads();
  for (int w = 1; w < PW; ++w) {
    if (ty == w)
#pragma unroll
      for (int l = 0; l < MC; ++l) {
        red[tx][l] = cadd(red[tx][l], accB[l]);
        redA[tx][l] = cadd(redA[tx][l], accA[l]);
      }
    __syncthreads();
  }
  // partA rows kb .. kb+63 of this column tile are contiguous
  const size_t baseA = ((size_t)blockIdx.x * (n + 1) + kb) * M;
  for (int idx = tid; idx < PT * M; idx += NT) {
    const int r = idx / M, i = idx % M;
    if (kb + r < n) partA[baseA + idx] = redA[r][i];
  }
  if (ty == 0 && jok) {
#pragma unroll
    for (int l = 0; l < MC; ++l)
      if (l < Lc) partB[((size_t)blockIdx.y * (n + 1) + j) * Lc + l] = red[tx][l];
  }
}

// Step 2: rho^A, rho^B from the tile partials (fixed order) and per-block
// partial sums over RB rows of the coupling coefficients
// c[i][l] = sum_k w_k varphi_l(k) rho^A[k][i] (eq. coefficients); the chain
// kernel adds up the blocks.  Each (row, channel) sum is one thread's; the
// coupling partials use every thread (pairs x row groups, combined in order).
constexpr int RB = 32;                   // rows per reduce block
constexpr int RT = RB * 16;              // threads per reduce block (>= 256 pairs)
template <typename T>
__global__ void __launch_bounds__(RT) k_cccs_reduce(int n, int ntiles, ChanTab<T> ch,
                                                     const v2<T>* __restrict__ partA,
                                                     const v2<T>* __restrict__ partB,
                                                     v2<T>* __restrict__ rhoA, v2<T>* __restrict__ rhoB,
                                                     v2<T>* __restrict__ partC) {
  __shared__ v2<T> ra[RB][16], wv[RB][16];
  __shared__ double pcr[RT], pci[RT];
  const int M = ch.M, Lc = ch.L, tid = threadIdx.x;
  const int kb = 1 + blockIdx.x * RB;
  {
    // item (row r, slot i): loads with clamped indices, 16 tiles at a time
    const int r = tid >> 4, i = tid & 15, k = kb + r;
    const int kc = k < n ? k : n - 1, ia = i < M ? i : M - 1, ib = i < Lc ? i : Lc - 1;
    const v2<T> w = ch.wvphi[(size_t)ib * (n + 1) + kc];
    v2<T> sa = mk<T>(0, 0), sb = mk<T>(0, 0);
    int t = 0;
    for (; t + 16 <= ntiles; t += 16) {
      v2<T> xa[16], xb[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        xa[u] = partA[((size_t)(t + u) * (n + 1) + kc) * M + ia];
        xb[u] = partB[((size_t)(t + u) * (n + 1) + kc) * Lc + ib];
      }
      // keep all 32 loads ahead of the sums (the scheduler would otherwise
      // wait for each load before issuing the next)
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        sa = cadd(sa, xa[u]);
        sb = cadd(sb, xb[u]);
      }
    }
    for (; t < ntiles; ++t) {
      sa = cadd(sa, partA[((size_t)t * (n + 1) + kc) * M + ia]);
      sb = cadd(sb, partB[((size_t)t * (n + 1) + kc) * Lc + ib]);
    }
    const bool row = k < n;
    if (row && i < M) rhoA[(size_t)k * M + i] = sa;
    if (row && i < Lc) rhoB[(size_t)k * Lc + i] = sb;
    ra[r][i] = (row && i < M) ? sa : mk<T>(0, 0);
    wv[r][i] = (row && i < Lc) ? w : mk<T>(0, 0);
  }
  __syncthreads();
  const int P = M * Lc;                      // <= 256 pairs
  const int G = RT / P;                      // row groups per pair
  const int pair = tid % P, grp = tid / P;
  if (grp < G) {
    const int i = pair / Lc, l = pair % Lc;
    double xr = 0, xi = 0;
    for (int r = grp; r < RB; r += G) {
      const v2<T> a = wv[r][l], b = ra[r][i];
      xr += (double)a.x * b.x - (double)a.y * b.y;
      xi += (double)a.x * b.y + (double)a.y * b.x;
    }
    pcr[grp * P + pair] = xr;
    pci[grp * P + pair] = xi;
  }
  __syncthreads();
  if (tid < P) {
    double xr = 0, xi = 0;
    for (int q = 0; q < G; ++q) {
      xr += pcr[q * P + tid];
      xi += pci[q * P + tid];
    }
    partC[(size_t)blockIdx.x * P + tid] = mk<T>((T)xr, (T)xi);
  }
}
int launch_cccs_reduce_blocks(int n) { return (n - 1 + RB - 1) / RB; }

// Block recurrences of the channel solves, one wave per recurrence.  A step
// is a small mat-vec with an Mr x Mr block A_q (Mr <= MC) and the previous
// step's vector.  The block is spread over the whole wave: lane = (row, part),
// PPR lanes per row, each holding EPL entries A_q[row][part + PPR e]; the
// vector entries come from LDS (one broadcast row), the row sums from DPP
// lane permutations inside each group of PPR lanes (no LDS round trip, no
// bpermute), and the part-0 lane of each row stores the result row.  Every
// lane works on every step, so a prefetch ring of PD steps in registers keeps
// the block loads PD steps ahead: step q reads ring slot q mod PD and refills
// it for step q + PD; the steps' scalars are read from LDS, so the ring is
// the only global load of a step.  LDS rows zs[l][0..MC) are zero beyond Mr.
template <int MC> struct LaneSplit {
  static constexpr int PPR = MC <= 8 ? MC : 64 / MC;            // lanes per row
  static constexpr int EPL = MC / PPR;                            // entries per lane
  static constexpr int PD = EPL == 1 ? 12 : (EPL <= 4 ? 6 : 2);   // prefetch ring depth
};

// v of lane l replaced by v of the lane the DPP control selects (within rows
// of 16 lanes); 64-bit values move as two 32-bit halves
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
// sum over each group of PPR consecutive lanes (PPR = 2, 4 or 8), in every lane
template <int PPR, typename T>
__device__ __forceinline__ v2<T> group_sum(v2<T> v) {
  if (PPR >= 2) v = mk<T>(v.x + dpp_mov<0xB1>(v.x), v.y + dpp_mov<0xB1>(v.y));     // lane ^ 1
  if (PPR >= 4) v = mk<T>(v.x + dpp_mov<0x4E>(v.x), v.y + dpp_mov<0x4E>(v.y));     // lane ^ 2
  if (PPR >= 8) v = mk<T>(v.x + dpp_mov<0x141>(v.x), v.y + dpp_mov<0x141>(v.y));   // 7 - lane in 8
  return v;
}

template <typename T, int EPL> struct StepEnt {
  v2<T> a[EPL];
};

// entries A[idx][row][part + PPR e] with clamped indices (rows beyond Mr
// repeat row Mr-1, columns beyond Mr repeat column Mr-1 and meet zero vector
// entries), so no loaded value is masked
template <typename T, int MC>
__device__ __forceinline__ void load_ent(StepEnt<T, LaneSplit<MC>::EPL>& r, const v2<T>* __restrict__ A, int Mr,
                                         int row, int part, int idx) {
  constexpr int PPR = LaneSplit<MC>::PPR, EPL = LaneSplit<MC>::EPL;
  const int rr = row < Mr ? row : Mr - 1;
  const v2<T>* Ar = A + ((size_t)idx * Mr + rr) * Mr;
#pragma unroll
  for (int e = 0; e < EPL; ++e) {
    const int m = part + PPR * e;
    r.a[e] = Ar[m < Mr ? m : Mr - 1];
  }
}

// One sweep over zs[0..len) (LDS, MC entries per row).
//   FWD (chain forward, PRE):  step q on row q with block base+q:
//        z_q = A_q (zs_q - c_q z_{q-1})      (zs_q holds the right-hand side)
//   FWD (interface forward):   z_q = zs_q - A_q z_{q-1}   (no product at q = 0)
//   !FWD: step q on row l = len-2-q with block base+l:
//        z_l = zs_l - c_l A_l z_{l+1}        (c = 1 unless HASC)
// cs: the steps' scalars in LDS, indexed by row (HASC).
template <typename T, int MC, bool FWD, bool PRE, bool HASC>
__device__ __forceinline__ void lds_sweep(v2<T>* zs, int len, const v2<T>* __restrict__ A, const v2<T>* cs,
                                          int base, int Mr) {
  constexpr int PPR = LaneSplit<MC>::PPR, EPL = LaneSplit<MC>::EPL, PD = LaneSplit<MC>::PD;
  const int lane = threadIdx.x, row = lane / PPR, part = lane % PPR;
  const bool writer = part == 0 && row < Mr;
  const int nsteps = FWD ? len : len - 1;
  if (nsteps <= 0) return;
  auto blk = [&](int q) {
    const int qc = q < nsteps ? q : nsteps - 1;
    return base + (FWD ? qc : len - 2 - qc);
  };
  StepEnt<T, EPL> R[PD];
#pragma unroll
  for (int d = 0; d < PD; ++d) load_ent<T, MC>(R[d], A, Mr, row, part, blk(d));
  for (int q0 = 0; q0 < nsteps; q0 += PD) {
#pragma unroll
    for (int d = 0; d < PD; ++d) {
      const int q = q0 + d;
      if (q < nsteps) {
        const int l = FWD ? q : len - 2 - q;
        const v2<T>* zl = zs + l * MC;
        const v2<T>* zp = zs + (FWD ? l - 1 : l + 1) * MC;
        v2<T> acc = mk<T>(0, 0);
        if (FWD && PRE) {
          const v2<T> c = cs[l];
#pragma unroll
          for (int e = 0; e < EPL; ++e) {
            const int m = part + PPR * e;
            const v2<T> x = q > 0 ? csub(zl[m], cmul(c, zp[m])) : zl[m];
            acc = cfma(acc, R[d].a[e], x);
          }
        } else if (!FWD || q > 0) {
#pragma unroll
          for (int e = 0; e < EPL; ++e) acc = cfma(acc, R[d].a[e], zp[part + PPR * e]);
        }
        acc = group_sum<PPR, T>(acc);
        v2<T> z;
        if (FWD && PRE) {
          z = acc;
        } else {
          const v2<T> b = zl[row < MC ? row : 0];
          z = (FWD && q == 0) ? b : csub(b, HASC ? cmul(cs[l], acc) : acc);
        }
        if (writer) zs[l * MC + row] = z;
        __syncthreads();                   // one wave: orders the row write before the next reads
        load_ent<T, MC>(R[d], A, Mr, row, part, blk(q + PD));
      }
    }
  }
}

// Step 3: channel right-hand sides, chunk-local block LU solves and the
// chunks' contributions to the interface right-hand sides.  Block = one wave;
// blockIdx.x = chunk, blockIdx.y = system (0: A, functions of x2 with the x1
// channels; 1: B, functions of x1 with the x2 channels).  Right-hand sides
// (Remark 4 convention):
//   r^A_i(k) = rho^A_i(k) - sum_{l > i} c_il varphi_l(k)
//   r^B_l(j) = rho^B_l(j) - sum_{m >= l} c_ml phi_m(j)
// Chunk rows s..e with the precomputed block LU (G_t = Schur-complement
// inverses, scalar couplings lo_t, up_t):
//   forward   Z_t = G_t (r_t - lo_t Z_{t-1})
//   backward  g_t = Z_t - up_t G_t g_{t+1},  g_e = Z_e
// The chunk lives in dynamic LDS (len x MC values).
template <typename T, int MC>
__global__ void __launch_bounds__(64) k_cccs_chain(ChanSys<T> SA, ChanSys<T> SB, ChanTab<T> ch,
                                                   int n, const v2<T>* __restrict__ rhoA,
                                                   const v2<T>* __restrict__ rhoB,
                                                   const v2<T>* __restrict__ partC, int nparts,
                                                   v2<T>* __restrict__ gA, v2<T>* __restrict__ gB,
                                                   v2<T>* __restrict__ HA, v2<T>* __restrict__ HB, int maxlen) {
  extern __shared__ __align__(16) unsigned char chain_lds[];
  v2<T>* zs = reinterpret_cast<v2<T>*>(chain_lds);       // [maxlen][MC]
  v2<T>* slo = zs + (size_t)maxlen * MC;                   // [maxlen] lo_t of the chunk rows
  v2<T>* sup = slo + maxlen;                               // [maxlen] up_t
  const bool isA = blockIdx.y == 0;
  const ChanSys<T>& S = isA ? SA : SB;
  const int p = blockIdx.x;
  if (p >= S.P) return;
  const int M = S.M, Mo = isA ? ch.L : ch.M;
  const int s = S.start[p], e = S.start[p + 1] - 1, len = e - s + 1;
  const int lane = threadIdx.x;
  v2<T>* g = isA ? gA : gB;
  const v2<T>* rho = isA ? rhoA : rhoB;
  // coupling coefficients c[i][l]: the reduce kernel's per-block partials,
  // added in a fixed order (16 loads in flight per lane, four partial sums)
  __shared__ v2<T> coef[256];
  const int npair = ch.M * ch.L;
  for (int idx = lane; idx < npair; idx += 64) {
    double xr[4] = {0, 0, 0, 0}, xi[4] = {0, 0, 0, 0};
    int b = 0;
    for (; b + 16 <= nparts; b += 16) {
      v2<T> c[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) c[u] = partC[(size_t)(b + u) * npair + idx];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        xr[u & 3] += c[u].x;
        xi[u & 3] += c[u].y;
      }
    }
    for (; b < nparts; ++b) {
      const v2<T> c = partC[(size_t)b * npair + idx];
      xr[0] += c.x;
      xi[0] += c.y;
    }
    coef[idx] = mk<T>((T)((xr[0] + xr[1]) + (xr[2] + xr[3])), (T)((xi[0] + xi[1]) + (xi[2] + xi[3])));
  }
  __syncthreads();
  // (a) right-hand sides of the chunk rows into LDS (zero beyond M).  Loads
  // use clamped indices and unused terms get a zero coefficient, so that all
  // loads of two elements per lane are in flight together.
  const v2<T>* basis = isA ? ch.vphi : ch.phi;
  for (int idx0 = 0; idx0 < len * MC; idx0 += 128) {
    v2<T> v[2], bs[2][MC];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int idx = idx0 + u * 64 + lane;
      const int q = idx < len * MC ? idx / MC : 0, i = idx % MC, node = s + q + 1;
      v[u] = rho[(size_t)node * M + (i < M ? i : M - 1)];
#pragma unroll
      for (int l = 0; l < MC; ++l) bs[u][l] = basis[(size_t)(l < Mo ? l : Mo - 1) * (n + 1) + node];
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int idx = idx0 + u * 64 + lane;
      if (idx < len * MC) {
        const int i = idx % MC;
        v2<T> r = mk<T>(0, 0);
        if (i < M) {
          r = v[u];
#pragma unroll
          for (int l = 0; l < MC; ++l) {
            const bool use = l < Mo && (isA ? (l > i) : (l >= i));
            const v2<T> cf = use ? (isA ? coef[i * Mo + l] : coef[l * M + i]) : mk<T>(0, 0);
            r = csub(r, cmul(cf, bs[u][l]));
          }
        }
        zs[idx] = r;
      }
    }
  }
  __syncthreads();
  for (int q = lane; q < len; q += 64) {
    slo[q] = S.lo[s + q];
    sup[q] = S.up[s + q];
  }
  __syncthreads();
  // (b) forward sweep, (c) backward sweep
  lds_sweep<T, MC, true, true, true>(zs, len, S.G, slo, s, M);
  lds_sweep<T, MC, false, false, true>(zs, len, S.G, sup, s, M);
  for (int idx = lane; idx < len * M; idx += 64) {
    const int q = idx / M, i = idx % M;
    g[(size_t)(s + q) * M + i] = zs[q * MC + i];
  }
  // (d) this chunk's contributions to the interface right-hand sides:
  //     interface p   from the last row:  Rinv_p     [g_e; 0]
  //     interface p-1 from the first row: Rinv_{p-1} [0; g_s]
  const int Q = S.P - 1;
  if (Q <= 0) return;
  const int R = 2 * M;
  v2<T>* H = isA ? HA : HB;           // [Q][2][R]: halves of Rinv_q [g(e_q); g(s_{q+1})]
  // (zs entries beyond M are zero, so clamped loads need no masking)
  if (lane < R) {
    v2<T> r1[MC], r2[MC];
    const v2<T>* Ri1 = S.Rinv + (size_t)(p < Q ? p : 0) * R * R + (size_t)lane * R;
    const v2<T>* Ri2 = S.Rinv + (size_t)(p > 0 ? p - 1 : 0) * R * R + (size_t)lane * R + M;
#pragma unroll
    for (int m = 0; m < MC; ++m) {
      r1[m] = Ri1[m < M ? m : M - 1];
      r2[m] = Ri2[m < M ? m : M - 1];
    }
    if (p < Q) {
      v2<T> acc = mk<T>(0, 0);
#pragma unroll
      for (int m = 0; m < MC; ++m) acc = cfma(acc, r1[m], zs[(len - 1) * MC + m]);
      H[((size_t)p * 2) * R + lane] = acc;
    }
    if (p > 0) {
      v2<T> acc = mk<T>(0, 0);
#pragma unroll
      for (int m = 0; m < MC; ++m) acc = cfma(acc, r2[m], zs[m]);
      H[((size_t)(p - 1) * 2 + 1) * R + lane] = acc;
    }
  }
}

// Step 3b: the interface system of each system (block tridiagonal in 2M x 2M
// blocks).  Its block Thomas sweeps (Rlo = Rinv Sub, Rup = Rinv Sup) are
// linear in the right-hand side, so the host applies them to unit vectors
// once per energy; here they act as one matrix, Y = Tif h with
// h_q = H_q^0 + H_q^1.  One wave per row of each system (blockIdx.y), lanes
// over the columns, the row sum by shuffles.  The block first issues its
// rows' Tif loads (up to 64 U columns per row in one round), then stages h
// (formed in FP64) in LDS from the small H vector, so that HBM sees only Tif.
constexpr int IF_MAXQR = 63 * 32;   // (P - 1) 2M for P <= 64 chunks and M <= 16
template <typename T>
__global__ void __launch_bounds__(256) k_cccs_iface_mv(ChanSys<T> SA, ChanSys<T> SB, v2<T>* __restrict__ YA,
                                                       v2<T>* __restrict__ YB, const v2<T>* __restrict__ HA,
                                                       const v2<T>* __restrict__ HB) {
  __shared__ v2<double> hs[IF_MAXQR];
  const bool isA = blockIdx.y == 0;
  const ChanSys<T>& S = isA ? SA : SB;
  const int R = 2 * S.M, QR = (S.P - 1) * R;
  const int row0 = blockIdx.x * 4;
  if (row0 >= QR) return;                        // the whole block: no barrier is left waiting
  const int row = row0 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  const bool rok = row < QR;
  const v2<T>* H = isA ? HA : HB;
  const v2<T>* Tr = S.Tif + (size_t)(rok ? row : QR - 1) * QR;
  constexpr int U = 12;                          // columns per lane in flight
  constexpr int NS = (IF_MAXQR + 255) / 256;     // staged entries per thread at most
  v2<T> t[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int c = lane + 64 * u;
    t[u] = Tr[c < QR ? c : QR - 1];
  }
  v2<T> h0[NS], h1[NS];
#pragma unroll
  for (int q = 0; q < NS; ++q) {
    const int c = threadIdx.x + 256 * q, cc = c < QR ? c : QR - 1, b = cc / R, i = cc - b * R;
    h0[q] = H[((size_t)b * 2) * R + i];
    h1[q] = H[((size_t)b * 2 + 1) * R + i];
  }
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int q = 0; q < NS; ++q) {
    const int c = threadIdx.x + 256 * q;
    if (c < QR) {
      v2<double> h;
      h.x = (double)h0[q].x + (double)h1[q].x;
      h.y = (double)h0[q].y + (double)h1[q].y;
      hs[c] = h;
    }
  }
  __syncthreads();
  double sr = 0, si = 0;
  for (int c0 = lane; c0 < QR; c0 += 64 * U) {
    if (c0 != lane) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int c = c0 + 64 * u;
        t[u] = Tr[c < QR ? c : QR - 1];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int c = c0 + 64 * u;
      if (c < QR) {
        const v2<double> h = hs[c];
        sr += (double)t[u].x * h.x - (double)t[u].y * h.y;
        si += (double)t[u].x * h.y + (double)t[u].y * h.x;
      }
    }
  }
  sr = wave_sum(sr);
  si = wave_sum(si);
  if (rok && lane == 0) (isA ? YA : YB)[row] = mk<T>((T)sr, (T)si);
}

// Step 4: retrieval e_t = g_t - V_t T_{p+1} - W_t B_{p-1}; thread per (t, i).
// MC bounds the channel count at compile time, so that every load of a group
// of G channels (spike entries and interface values of both terms) is issued
// before the first use (clamped indices; unused terms are skipped at the
// arithmetic: a group's T terms, then its B terms, one group for M <= 8).
// One-wave blocks spread the few rows over every CU.
template <typename T, int MC>
__global__ void __launch_bounds__(64) k_cccs_retrieve(ChanSys<T> SA, ChanSys<T> SB,
                                                      const v2<T>* __restrict__ gA,
                                                      const v2<T>* __restrict__ gB,
                                                      const v2<T>* __restrict__ YA,
                                                      const v2<T>* __restrict__ YB,
                                                      v2<T>* __restrict__ eA, v2<T>* __restrict__ eB) {
  constexpr int G = MC < 8 ? MC : 8;
  const bool isA = blockIdx.y == 0;
  const ChanSys<T>& S = isA ? SA : SB;
  const int M = S.M, MM = M * M, R = 2 * M;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= S.N * M) return;
  const int t = idx / M, i = idx % M;
  const v2<T>* g = isA ? gA : gB;
  const v2<T>* Y = isA ? YA : YB;
  v2<T>* e = isA ? eA : eB;
  // chunk of row t: start[p] = floor(N p / P), so p = floor(t P / N) or p + 1
  // (the boundary is recomputed rather than loaded: no load ahead of the rest)
  int p = (int)(((long long)t * S.P) / S.N);
  if (p + 1 < S.P && t >= (int)(((long long)S.N * (p + 1)) / S.P)) ++p;
  const bool hasT = p + 1 < S.P, hasB = p > 0;
  const size_t base = (size_t)t * MM + (size_t)i * M;
  // Y holds P 2M-blocks, so both clamped interface rows stay inside it
  const v2<T>* Tn = Y + (size_t)p * R + M;
  const v2<T>* Bp = Y + (size_t)(hasB ? p - 1 : 0) * R;
  const v2<T>* Sr[2] = {S.Vs + base, S.Ws + base};
  const v2<T>* Xr[2] = {Tn, Bp};
  const bool on[2] = {hasT, hasB};
  v2<T> v = g[(size_t)t * M + i];
#pragma unroll
  for (int m0 = 0; m0 < MC; m0 += G) {
    v2<T> sv[2][G], xv[2][G];                    // [0]: V_t, T_{p+1}; [1]: W_t, B_{p-1}
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int u = 0; u < G; ++u) {
        const int mc = m0 + u < M ? m0 + u : M - 1;
        sv[h][u] = Sr[h][mc];
        xv[h][u] = Xr[h][mc];
      }
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int u = 0; u < G; ++u)
        if (on[h] && m0 + u < M) v = csub(v, cmul(sv[h][u], xv[h][u]));
  }
  e[(size_t)(t + 1) * M + i] = v;   // node index t+1
}

// Step 5: expansion u += sum_m eA[k][m] phi_m(j) + sum_l eB[j][l] varphi_l(k).
// The row-dependent factors of the block's SY * ROWS rows are staged in LDS
// (one load each), the column-dependent ones stay in registers.
template <typename T, int MC>
__global__ void __launch_bounds__(256) k_cccs_expand(int n, int pitch, v2<T>* __restrict__ u,
                                                     ChanTab<T> ch, const v2<T>* __restrict__ eA,
                                                     const v2<T>* __restrict__ eB) {
  constexpr int BR = SY * ROWS;
  static_assert(BR * MC <= SX * SY, "one staged factor per thread");
  __shared__ v2<T> ea[BR][MC], vp[BR][MC];
  __shared__ v2<T> ebt[MC][SX + 1];              // eB of the block's columns, transposed (odd pitch: the
                                                 // transposing writes avoid bank conflicts)
  const int tid = threadIdx.x + SX * threadIdx.y;
  const int kb = 1 + blockIdx.y * BR;
  const int M = ch.M, Lc = ch.L;
  const int j = 1 + blockIdx.x * SX + threadIdx.x;
  const bool jok = j < n;
  const int jc = jok ? j : n - 1;
  // every load first (clamped indices, selects afterwards): the thread's rows
  // of u, its column factors, one staged row factor
  v2<T> uv[ROWS];
#pragma unroll
  for (int q = 0; q < ROWS; ++q) {
    const int k = kb + threadIdx.y * ROWS + q;
    uv[q] = u[(size_t)(k < n ? k : n - 1) * pitch + jc];
  }
  v2<T> ph[MC];
#pragma unroll
  for (int m = 0; m < MC; ++m) ph[m] = ch.phi[(size_t)(m < M ? m : M - 1) * (n + 1) + jc];
  // eB[j][l] of the block's SX columns is contiguous: coalesced loads, then
  // transposed through LDS (a per-column load would touch one line per lane)
  constexpr int NEB = (SX * MC + SX * SY - 1) / (SX * SY);
  const int jb = 1 + blockIdx.x * SX;
  v2<T> ebl[NEB];
#pragma unroll
  for (int q = 0; q < NEB; ++q) {
    const int idx = tid + SX * SY * q, cj = jb + idx / Lc;
    ebl[q] = eB[(size_t)(cj < n ? cj : n - 1) * Lc + idx % Lc];
  }
  const int sr = tid / MC, sm = tid % MC, sk = kb + sr, skc = sk < n ? sk : n - 1;
  v2<T> sa = mk<T>(0, 0), sv = mk<T>(0, 0);
  if (tid < BR * MC) {
    sa = eA[(size_t)skc * M + (sm < M ? sm : M - 1)];
    sv = ch.vphi[(size_t)(sm < Lc ? sm : Lc - 1) * (n + 1) + skc];
  }
  __builtin_amdgcn_sched_barrier(0);
  if (tid < BR * MC) {
    ea[sr][sm] = (sk < n && sm < M) ? sa : mk<T>(0, 0);
    vp[sr][sm] = (sk < n && sm < Lc) ? sv : mk<T>(0, 0);
  }
#pragma unroll
  for (int q = 0; q < NEB; ++q) {
    const int idx = tid + SX * SY * q;
    if (idx < SX * Lc) ebt[idx % Lc][idx / Lc] = ebl[q];
  }
  for (int idx = tid; idx < SX * (MC - Lc); idx += SX * SY)                // unused channels
    ebt[Lc + idx / SX][idx % SX] = mk<T>(0, 0);
#pragma unroll
  for (int m = 0; m < MC; ++m)
    if (m >= M) ph[m] = mk<T>(0, 0);
  __syncthreads();
  if (!jok) return;
  v2<T> eb[MC];
#pragma unroll
  for (int m = 0; m < MC; ++m) eb[m] = ebt[m][threadIdx.x];
#pragma unroll
  for (int q = 0; q < ROWS; ++q) {
    const int r = threadIdx.y * ROWS + q, k = kb + r;
    if (k >= n) break;
    v2<T> v = uv[q];
#pragma unroll
    for (int m = 0; m < MC; ++m) {
      v = cfma(v, ea[r][m], ph[m]);
      v = cfma(v, eb[m], vp[r][m]);
    }
    u[(size_t)k * pitch + j] = v;
  }
}

// ----------------------------------------------------------------------------
// Vector kernels for the FP64 outer loop (grid-stride over interior nodes).
// Interior-node loop of the vector kernels: 256-thread blocks = 64 columns x
// 4 row groups; blockIdx.x selects a 64-column tile, blockIdx.y strides the
// rows.  No integer division; independent rows are unrolled so that their
// loads are in flight together.
#define MGC_NODE_LOOP(n, k, j)                                                  \
  const int j = 1 + (int)blockIdx.x * 64 + ((int)threadIdx.x & 63);             \
  const int k##_first = 1 + (int)blockIdx.y * 4 + ((int)threadIdx.x >> 6);      \
  const int k##_step = (int)gridDim.y * 4;                                      \
  if (j < (n))                                                                  \
    _Pragma("unroll 4") for (int k = k##_first; k < (n); k += k##_step)
__device__ __forceinline__ int flat_block() { return blockIdx.x + gridDim.x * blockIdx.y; }

// ----------------------------------------------------------------------------
// FGMRES bookkeeping on the device, by one block after the reductions
// finished.  Loads go to LDS in parallel; only the short sequential Givens
// arithmetic runs on one thread.
template <int NT>
__device__ void gmres_step_blk(const GmresState& st, int j, int m, double tol_abs, const double* __restrict__ part,
                               int nb, int ps) {
  // after the final norm: column j of H (= projections, then the norm),
  // earlier rotations, new rotation, residual estimate.  The state loads are
  // issued together with the norm's partial loads (nb partials, ps apart).
  __shared__ double col[2 * 34], rot[4 * 33], gg[4], red[NT / 64];
  const int tid = threadIdx.x + blockDim.x * threadIdx.y;
  const int R = m + 1;
  double h0 = 0, h1 = 0, r0 = 0, r1 = 0, r2 = 0, r3 = 0, g0 = 0, g1 = 0;
  if (tid <= j) {
    h0 = st.hcol[2 * tid];
    h1 = st.hcol[2 * tid + 1];
  }
  if (tid < j) {
    r0 = st.cs[2 * tid];
    r1 = st.cs[2 * tid + 1];
    r2 = st.sn[2 * tid];
    r3 = st.sn[2 * tid + 1];
  }
  if (tid == 0) {
    g0 = st.g[2 * j];
    g1 = st.g[2 * j + 1];
  }
  // ||Y||^2: the partials strided over the threads, wave sums added in
  // wave order
  double s = 0.0;
  for (int b = tid; b < nb; b += NT) s += part[(size_t)b * ps];
  s = wave_sum(s);
  if ((tid & 63) == 0) red[tid >> 6] = s;
  if (tid <= j) {
    col[2 * tid] = h0;
    col[2 * tid + 1] = h1;
  }
  if (tid < j) {
    rot[4 * tid] = r0;
    rot[4 * tid + 1] = r1;
    rot[4 * tid + 2] = r2;
    rot[4 * tid + 3] = r3;
  }
  __syncthreads();
  if (tid == 0) {
    double nrm2 = 0.0;
    for (int w = 0; w < NT / 64; ++w) nrm2 += red[w];
    st.nrm2[0] = nrm2;
    gg[0] = g0;
    gg[1] = g1;
    gg[2] = sqrt(nrm2);
    const double nrm = gg[2];
    col[2 * (j + 1)] = nrm;
    col[2 * (j + 1) + 1] = 0.0;
    for (int i = 0; i < j; ++i) {
      const double cr = rot[4 * i], ci = rot[4 * i + 1], sr = rot[4 * i + 2], si = rot[4 * i + 3];
      const double a = col[2 * i], b = col[2 * i + 1], c = col[2 * i + 2], d = col[2 * i + 3];
      // t1 = conj(cs) x1 + conj(sn) x2 ; t2 = -sn x1 + cs x2
      col[2 * i] = cr * a + ci * b + sr * c + si * d;
      col[2 * i + 1] = cr * b - ci * a + sr * d - si * c;
      col[2 * i + 2] = -(sr * a - si * b) + (cr * c - ci * d);
      col[2 * i + 3] = -(sr * b + si * a) + (cr * d + ci * c);
    }
    const double hr = col[2 * j], hi = col[2 * j + 1], nr = col[2 * j + 2], ni = col[2 * j + 3];
    const double den = sqrt(hr * hr + hi * hi + nr * nr + ni * ni);
    const double cr = hr / den, ci = hi / den, sr = nr / den, si = ni / den;
    st.cs[2 * j] = cr; st.cs[2 * j + 1] = ci; st.sn[2 * j] = sr; st.sn[2 * j + 1] = si;
    col[2 * j] = den; col[2 * j + 1] = 0; col[2 * j + 2] = 0; col[2 * j + 3] = 0;
    const double gr = gg[0], gi = gg[1];
    // g_{j+1} = -sn g_j ; g_j = conj(cs) g_j
    const double g1r = -(sr * gr - si * gi), g1i = -(sr * gi + si * gr);
    st.g[2 * (j + 1)] = g1r;
    st.g[2 * (j + 1) + 1] = g1i;
    st.g[2 * j] = cr * gr + ci * gi;
    st.g[2 * j + 1] = cr * gi - ci * gr;
    const double est = sqrt(g1r * g1r + g1i * g1i);
    st.est[j] = est;
    st.scale[j + 1] = nrm > 0 ? 1.0 / nrm : 0.0;
    if (st.kstar[0] < 0 && (est <= tol_abs || !(nrm > 0))) st.kstar[0] = j + 1;
  }
  __syncthreads();
  if (tid <= j + 1) {                  // Hessenberg is column-major (m+1) x m complex
    st.H[2 * (j * R + tid)] = col[2 * tid];
    st.H[2 * (j * R + tid) + 1] = col[2 * tid + 1];
  }
}

// Least squares of the cycle (one block of NT threads, after its last Givens
// step): y = H(1:k,1:k)^{-1} g(1:k); k = first step meeting the tolerance,
// else the mm <= m steps the cycle performed; update coefficients y_i.  H and
// g are staged in LDS by all threads, the back substitution runs on one thread.
template <int NT>
__device__ void gmres_solve_blk(const GmresState& st, int m, int mm) {
  __shared__ double Hs[2 * 33 * 32], gs[2 * 33], ys[2 * 32];
  const int tid = threadIdx.x + blockDim.x * threadIdx.y;
  const int R = m + 1;
  __syncthreads();                     // the block's own H and g stores are done
  for (int q = tid; q < 2 * R * m; q += NT) Hs[q] = st.H[q];
  for (int q = tid; q < 2 * R; q += NT) gs[q] = st.g[q];
  __syncthreads();
  if (tid == 0) {
    const int k = (st.kstar[0] > 0 && st.kstar[0] <= mm) ? st.kstar[0] : mm;
    st.kused[0] = k;
    for (int i = k - 1; i >= 0; --i) {
      double vr = gs[2 * i], vi = gs[2 * i + 1];
      for (int c = i + 1; c < k; ++c) {
        const double hr = Hs[2 * (c * R + i)], hi = Hs[2 * (c * R + i) + 1];
        vr -= hr * ys[2 * c] - hi * ys[2 * c + 1];
        vi -= hr * ys[2 * c + 1] + hi * ys[2 * c];
      }
      const double dr = Hs[2 * (i * R + i)], di = Hs[2 * (i * R + i) + 1];
      const double den = dr * dr + di * di;
      ys[2 * i] = (vr * dr + vi * di) / den;
      ys[2 * i + 1] = (vi * dr - vr * di) / den;
    }
    for (int i = k; i < m; ++i) { ys[2 * i] = 0; ys[2 * i + 1] = 0; }
  }
  __syncthreads();
  if (tid < m) {
    st.y[2 * tid] = ys[2 * tid];
    st.y[2 * tid + 1] = ys[2 * tid + 1];
    st.upcoef[tid] = make_double2(ys[2 * tid], ys[2 * tid + 1]);
  }
}

// ----------------------------------------------------------------------------
// Fused Arnoldi passes of FGMRES step j (FP64 basis W_0..W_{J-1}, J = j+1,
// new vector Y = W_{j+1}), classical Gram-Schmidt with one re-orthogonalisation:
//   k_apply_dot  : Y = A z_j (exact operator)          per-block c_q = W_q^H Y
//   k_axpy_pass  : a_q = s_q^2 c_q, Y -= sum a_q W_q,   per-block c_q = W_q^H Y
//   k_reorth_step: same with the new c_q (pass 1),      per-block ||Y||^2,
//                  then ||Y||, Hessenberg column j and its Givens rotation
// The re-orthogonalisation is selective: the operator pass and pass 0 also
// accumulate ||Y||^2, and pass 1 skips its sweep (taking pass 0's norm)
// when pass 0 kept more than eta of the norm, since one classical pass then
// loses orthogonality only at the level of rounding / eta.
// Two sweeps of (J + 2) vectors per step, three with the second pass.
// s_q = 1/||W_q|| (unscaled basis).
// No pass finishes its own reduction: a per-block fence and ticket would cost
// far more than the kernel boundary, so each consumer adds up the producer's
// per-block partials itself (every block in the same fixed order; block 0
// also records the projections h_q += s_q c_q).
// The axpy passes run over the whole padded array: every basis vector is zero
// outside the interior (the workspace starts zeroed, the operator pass writes
// interior nodes only and the axpys keep zeros zero), so the ring and the
// padding add nothing to the dots.  J (<= 16) is a template argument, so that
// all loads of a node are issued together.
constexpr int AB = 512;          // threads per block of the Arnoldi passes
constexpr int AD_SY = 8;         // k_apply_dot block: 64 columns x 8 row groups
constexpr int AX_BLOCKS = 256;   // at most this many blocks per Arnoldi pass

#define MGC_JFOR(q) _Pragma("unroll") for (int q = 0; q < J; ++q)

// rows: rows per thread (each thread walks `rows` consecutive rows of a column)
template <typename TZ, int J>
__global__ void __launch_bounds__(AB) k_apply_dot(Level<double> L, const v2<TZ>* __restrict__ z,
                                                  const double2* __restrict__ W, size_t stride,
                                                  double2* __restrict__ Y, double* __restrict__ part,
                                                  int rows) {
  const int j = 1 + blockIdx.x * SX + threadIdx.x;
  const int k0 = 1 + (blockIdx.y * AD_SY + threadIdx.y) * rows;
  const int n = L.n, p = L.pitch;
  double acc[2 * J + 1];
#pragma unroll
  for (int q = 0; q <= 2 * J; ++q) acc[q] = 0.0;
  if (j < n) {
    ColumnStencil<double, v2<TZ>> cs(L, z, j, __builtin_amdgcn_readfirstlane(k0));
#pragma unroll 2
    for (int r = 0; r < rows; ++r) {
      const int k = __builtin_amdgcn_readfirstlane(k0 + r);
      if (k < n) {
        const size_t idx = (size_t)k * p + j;
        double2 w[J];
        MGC_JFOR(q) w[q] = W[q * stride + idx];
        const double2 o = cs.step(k);
        Y[idx] = o;
        MGC_JFOR(q) {
          acc[2 * q] += w[q].x * o.x + w[q].y * o.y;
          acc[2 * q + 1] += w[q].x * o.y - w[q].y * o.x;
        }
        acc[2 * J] += o.x * o.x + o.y * o.y;
      }
    }
  }
  double tot[2 * J + 1];
  block_sum<2 * J + 1>(acc, tot);
  if (threadIdx.x == 0 && threadIdx.y == 0) {
#pragma unroll
    for (int q = 0; q <= 2 * J; ++q) part[(size_t)flat_block() * (2 * J + 1) + q] = tot[q];
  }
}

// Flat axpy sweep over Nf = (n+1) * pitch nodes.  pin: nbin x (2J + 1)
// per-block dots and ||Y||^2 of the previous pass; pass 0 starts the
// projections h, pass 1 adds.  Pass 0 writes the new per-block dots and
// ||Y||^2, pass 1 (NORM) ||Y||^2 only, to pout.  Y32 (nullable): the new
// vector also rounded to FP32, unscaled (the FP32 cycle's input, same pitch).
template <int J, bool NORM>
__device__ __forceinline__ void axpy_sweep(size_t Nf, size_t stride, const double2* __restrict__ W,
                                           double2* __restrict__ Y, float2* __restrict__ Y32,
                                           const double* __restrict__ pin, int nbin,
                                           double* __restrict__ pout, const GmresState& st, int pass) {
  constexpr int NV = NORM ? 1 : 2 * J + 1;
  __shared__ double dsum[2 * J + 1];
  __shared__ double2 cf[J];
  finish_sum_nt<AB>(pin, nbin, 2 * J + 1, dsum);
  if (threadIdx.x < J) {
    const int i = threadIdx.x;
    const double s = st.scale[i], cr = dsum[2 * i], ci = dsum[2 * i + 1];
    cf[i] = make_double2(s * s * cr, s * s * ci);
    if (blockIdx.x == 0) {
      const double hr = pass == 0 ? 0.0 : st.hcol[2 * i], hi = pass == 0 ? 0.0 : st.hcol[2 * i + 1];
      st.hcol[2 * i] = hr + s * cr;
      st.hcol[2 * i + 1] = hi + s * ci;
    }
  }
  __syncthreads();
  double2 c[J];
  MGC_JFOR(q) c[q] = cf[q];
  double acc[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) acc[q] = 0.0;
  const size_t nt = (size_t)gridDim.x * AB;
#pragma unroll 2
  for (size_t i = (size_t)blockIdx.x * AB + threadIdx.x; i < Nf; i += nt) {
    double2 w[J];
    MGC_JFOR(q) w[q] = W[q * stride + i];
    double2 y = Y[i];
    MGC_JFOR(q) {
      y.x -= c[q].x * w[q].x - c[q].y * w[q].y;
      y.y -= c[q].x * w[q].y + c[q].y * w[q].x;
    }
    Y[i] = y;
    if (Y32) Y32[i] = make_float2((float)y.x, (float)y.y);
    if (NORM) {
      acc[0] += y.x * y.x + y.y * y.y;
    } else {
      MGC_JFOR(q) {
        acc[2 * q] += w[q].x * y.x + w[q].y * y.y;
        acc[2 * q + 1] += w[q].x * y.y - w[q].y * y.x;
      }
      acc[2 * J] += y.x * y.x + y.y * y.y;
    }
  }
  double tot[NV];
  block_sum<NV>(acc, tot);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) pout[(size_t)blockIdx.x * NV + q] = tot[q];
  }
}

template <int J>
__global__ void __launch_bounds__(AB) k_axpy_pass(size_t Nf, size_t stride, const double2* __restrict__ W,
                                                  double2* __restrict__ Y, float2* __restrict__ Y32,
                                                  const double* __restrict__ pin, int nbin,
                                                  double* __restrict__ pout, GmresState st) {
  axpy_sweep<J, false>(Nf, stride, W, Y, Y32, pin, nbin, pout, st, 0);
}

// Pass 1 and the Givens step in one launch (after the cycle's last step, the
// block that forms the column also solves the cycle's least squares).  Every block first decides from
// the ||Y||^2 partials of the operator pass (p0) and of pass 0 (pin) whether
// the second sweep is needed.  Usually it is not: then block 0 alone forms
// column j of H from pass 0's ||Y||^2 partials and the other blocks end at
// once.  Otherwise every block sweeps, and the block that finishes last (a
// device-scope fence and ticket per block, paid only on this rare path)
// forms the column from the sweep's partials and clears the ticket.
template <int J>
__global__ void __launch_bounds__(AB) k_reorth_step(size_t Nf, size_t stride, const double2* __restrict__ W,
                                                    double2* __restrict__ Y, float2* __restrict__ Y32,
                                                    const double* __restrict__ pin,
                                                    int nbin, double* __restrict__ pout, GmresState st,
                                                    const double* __restrict__ p0, int nb0, int j, int m,
                                                    int mm, double tol_abs, double eta) {
  __shared__ double nn[2];
  __shared__ int last;
  finish_sum_pair<AB>(pin + 2 * J, nbin, 2 * J + 1, p0 + 2 * J, nb0, 2 * J + 1, nn);
  if (nn[0] >= eta * eta * nn[1]) {
    // pass 0 kept enough of the norm: its ||Y||^2 partials are the result
    if (blockIdx.x == 0) {
      gmres_step_blk<AB>(st, j, m, tol_abs, pin + 2 * J, nbin, 2 * J + 1);
      if (j == mm - 1) gmres_solve_blk<AB>(st, m, mm);
    }
    return;
  }
  axpy_sweep<J, true>(Nf, stride, W, Y, Y32, pin, nbin, pout, st, 1);
  __threadfence();
  if (threadIdx.x == 0) last = atomicAdd(st.ticket, 1u) == gridDim.x - 1 ? 1 : 0;
  __syncthreads();
  if (!last) return;
  __threadfence();
  if (threadIdx.x == 0) st.ticket[0] = 0u;
  gmres_step_blk<AB>(st, j, m, tol_abs, pout, gridDim.x, 1);
  if (j == mm - 1) gmres_solve_blk<AB>(st, m, mm);
}
#undef MGC_JFOR

// u += sum_q coef_q Z_q with Z stored in precision TZ.
template <typename TZ, int JMAX>
__global__ void __launch_bounds__(256) k_update(int n, int pitch, size_t stride,
                                                const v2<TZ>* __restrict__ Z, int J,
                                                const double2* __restrict__ coef,
                                                double2* __restrict__ u) {
  __shared__ double2 cf[JMAX];
  if (threadIdx.x < J) cf[threadIdx.x] = coef[threadIdx.x];
  __syncthreads();
  MGC_NODE_LOOP(n, k, j) {
    const size_t idx = (size_t)k * pitch + j;
    double2 v = u[idx];
    for (int q = 0; q < J; ++q) {
      v2<double> z = cvt<double>(Z[q * stride + idx]);
      double2 c = cf[q];
      v.x += c.x * z.x - c.y * z.y;
      v.y += c.x * z.y + c.y * z.x;
    }
    u[idx] = v;
  }
}

// out = s * in with precision conversion; s read from the device (nullable = 1).
template <typename TI, typename TO>
__global__ void __launch_bounds__(256) k_scale_copy(int n, int pitch_in, int pitch_out,
                                                    const v2<TI>* __restrict__ in,
                                                    const double* __restrict__ s,
                                                    v2<TO>* __restrict__ out) {
  const double sc = s ? *s : 1.0;
  MGC_NODE_LOOP(n, k, j) {
    v2<TI> v = in[(size_t)k * pitch_in + j];
    out[(size_t)k * pitch_out + j] = mk<TO>((TO)(sc * v.x), (TO)(sc * v.y));
  }
}

// Weighted copy for the transpose solve: out = w_j w_k in  or in / (w_j w_k).
__global__ void __launch_bounds__(256) k_weight(int n, int pitch, const double2* __restrict__ w,
                                                int divide, const double2* __restrict__ in,
                                                double2* __restrict__ out) {
  MGC_NODE_LOOP(n, k, j) {
    v2<double> ww = cmul(w[j], w[k]);
    v2<double> v = in[(size_t)k * pitch + j];
    out[(size_t)k * pitch + j] = divide ? cdiv(v, ww) : cmul(v, ww);
  }
}

// Sum of per-block partials in fixed order: out[q] = sum_b part[b*nq + q];
// out[0] also lands in copy_to (nullable).
__global__ void __launch_bounds__(256) k_sum_partials(int nb, int nq, const double* __restrict__ part,
                                                      double* __restrict__ out, double* copy_to) {
  finish_sum(part, nb, nq, out);
  if (copy_to && threadIdx.x == 0) *copy_to = out[0];
}

// ----------------------------------------------------------------------------
// FGMRES bookkeeping on the device (single thread).  State layout in `st`
// (doubles):  see GmresState in launch.h.
// start of a restart cycle (one thread): beta = sqrt(nrm2), scale_0 = 1/beta,
// g = (beta, 0, ...)
__device__ void gmres_begin_thread(const GmresState& st, int m) {
  double beta = sqrt(st.nrm2[0]);
  st.scale[0] = beta > 0 ? 1.0 / beta : 0.0;
  for (int i = 0; i <= m; ++i) { st.g[2 * i] = 0; st.g[2 * i + 1] = 0; }
  st.g[0] = beta;
  st.kstar[0] = -1;
  st.beta[0] = beta;
}
__global__ void k_gmres_begin(GmresState st, int m) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  gmres_begin_thread(st, m);
}

// End of a restart cycle (one block of 256): ||r||^2 and ||f||^2 of the true
// residual from the residual pass's per-block partials (the fixed order of
// k_sum_partials) into scal[0..1] and ||r||^2 into the Krylov state, the
// host's report rep = (||r||^2, ||f||^2, steps used), then the next cycle's
// start.
__global__ void __launch_bounds__(256) k_cycle_end(int nb, const double* __restrict__ part,
                                                   double* __restrict__ scal, GmresState st, int m,
                                                   double* __restrict__ rep) {
  finish_sum(part, nb, 2, scal);
  if (threadIdx.x == 0) {
    st.nrm2[0] = scal[0];
    rep[0] = scal[0];
    rep[1] = scal[1];
    rep[2] = (double)st.kused[0];
    gmres_begin_thread(st, m);
  }
}

// Iterative refinement scale: s = sqrt(N)/||r|| (RMS normalisation) in sc[0];
// the complex coefficient (1/s, 0) in sc[2..3], 16-byte aligned for double2 loads.
__global__ void k_ir_scale(const double* nrm2, double Nn, double* sc) {
  double r = sqrt(nrm2[0]);
  double s = r > 0 ? sqrt(Nn) / r : 1.0;
  sc[0] = s;
  sc[2] = 1.0 / s;
  sc[3] = 0.0;
}
__global__ void k_copy_scalar(const double* src, double* dst) { dst[0] = src[0]; }
__global__ void k_fill_zero(size_t n16, double2* p) {
  for (size_t i = blockIdx.x * 256 + threadIdx.x; i < n16; i += (size_t)gridDim.x * 256) p[i] = make_double2(0, 0);
}

// ----------------------------------------------------------------------------
// Right-hand side of the Temkin-Poet impact problem (real region only).
__global__ void __launch_bounds__(256) k_rhs_tp(int n, int pitch, int j0, const double2* __restrict__ z,
                                                double Z1, double Z2, double lam, double k0,
                                                double2* __restrict__ chi) {
  const double pref = 2.0 * Z1 * sqrt(Z1);
  MGC_NODE_LOOP(n, k, j) {
    double v = 0.0;
    // chi0(k, j) + chi0(j, k); z is real on nodes <= j0
    if (k <= j0 && j <= j0) {
      const double xj = z[j].x, xk = z[k].x;
      const double xm = j > k ? xj : xk;
      const double c1 = (lam / xm - Z2 / xk) * pref * xj * exp(-Z1 * xj) * sin(k0 * xk);
      const double c2 = (lam / xm - Z2 / xj) * pref * xk * exp(-Z1 * xk) * sin(k0 * xj);
      v = (c1 + c2) * 0.70710678118654752440;
    }
    chi[(size_t)k * pitch + j] = make_double2(v, 0.0);
  }
}

// zeta partials: sum t_j t_k phik1_j phik2_k (chi - V12 u)  over the real region.
__global__ void __launch_bounds__(256) k_zeta_part(int n, int pitch, int j0, const double2* __restrict__ tm,
                                                   const double* __restrict__ f1,
                                                   const double* __restrict__ f2,
                                                   const double2* __restrict__ u,
                                                   const double2* __restrict__ chi,
                                                   double* __restrict__ part) {
  double acc[2] = {0, 0};
  MGC_NODE_LOOP(n, k, j) {
    if (k > j0 || j > j0) continue;
    const size_t idx = (size_t)k * pitch + j;
    v2<double> v12 = tm[j > k ? j : k];
    v2<double> src = csub(chi[idx], cmul(v12, u[idx]));
    const double wgt = f1[j] * f2[k];
    acc[0] += wgt * src.x;
    acc[1] += wgt * src.y;
  }
  double tot[2];
  block_sum<2>(acc, tot);
  if (threadIdx.x == 0) { part[2 * flat_block()] = tot[0]; part[2 * flat_block() + 1] = tot[1]; }
}


// Many momentum pairs at once (eq. double-ionization for each pair a):
//   zeta_a = sum_k f2_a[k] sum_j s[k][j] f1_a[j],   s = chi - V12 u,
// over the real region, rows and columns 1 .. top.  Block = SWR rows k and one
// of SWJ column ranges, thread = pair a (blockDim.x = pp).  s of the block's
// rows is staged in LDS SWC columns at a time (one value per thread and
// round), the test functions are read as [node][pair] rows, coalesced over the
// pairs, a round's SWC of them issued together.  One (re, im) partial per
// block and pair; k_zeta_sweep_sum adds the blocks in a fixed order.
constexpr int SWR = 8, SWJ = 8, SWC = 32;
__global__ void __launch_bounds__(256) k_zeta_sweep_part(int n, int pitch, int top, int pp,
                                                         const double2* __restrict__ tm,
                                                         const double* __restrict__ F1T,
                                                         const double* __restrict__ F2T,
                                                         const double2* __restrict__ u,
                                                         const double2* __restrict__ chi,
                                                         double* __restrict__ part) {
  __shared__ v2<double> st[SWR][SWC];
  const int a = threadIdx.x;
  const int k0 = 1 + blockIdx.x * SWR;
  const int jn = (top + SWJ - 1) / SWJ;
  const int jb = 1 + blockIdx.y * jn, je = jb + jn < top + 1 ? jb + jn : top + 1;   // j in [jb, je)
  double ar[SWR], ai[SWR];
#pragma unroll
  for (int r = 0; r < SWR; ++r) ar[r] = ai[r] = 0.0;
  for (int c0 = jb; c0 < je; c0 += SWC) {
    double f[SWC];
#pragma unroll
    for (int c = 0; c < SWC; ++c) {
      const int j = c0 + c;
      f[c] = F1T[(size_t)(j < n ? j : n) * pp + a];
    }
    for (int q = a; q < SWR * SWC; q += pp) {
      const int r = q / SWC, c = q - r * SWC, k = k0 + r, j = c0 + c;
      v2<double> v = mk<double>(0, 0);
      if (k <= top && j < je) {
        const size_t idx = (size_t)k * pitch + j;
        v = csub(chi[idx], cmul(tm[j > k ? j : k], u[idx]));
      }
      st[r][c] = v;
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < SWC; ++c)
#pragma unroll
      for (int r = 0; r < SWR; ++r) {
        const v2<double> sv = st[r][c];      // zero beyond the column range
        ar[r] += sv.x * f[c];
        ai[r] += sv.y * f[c];
      }
    __syncthreads();
  }
  double zr = 0.0, zi = 0.0;
#pragma unroll
  for (int r = 0; r < SWR; ++r) {
    const int k = k0 + r;
    if (k <= top) {
      const double w = F2T[(size_t)k * pp + a];
      zr += w * ar[r];
      zi += w * ai[r];
    }
  }
  const size_t blk = blockIdx.x + (size_t)gridDim.x * blockIdx.y;
  part[blk * 2 * pp + 2 * a] = zr;
  part[blk * 2 * pp + 2 * a + 1] = zi;
}

// Weighted test functions of the sweep (eq. testfunction), one thread per
// function: column c < pp of F takes momentum kk[c] (the x1 side), column
// pp + c momentum kk[npairs + c] (the x2 side); the table is [side][node][pair],
// F[(side (n+1) + j) pp + c].  The three-point finite-difference recurrence of
// the real-axis radial equation starts from phi(0) = 0, phi(h) = h; the
// amplitude is fixed by the WKB-type matching at node jr = min(j0, top - 1)
// (unit asymptotic amplitude 1 / sqrt(p)), and the trapezoid weight (h, half
// at j0) is folded in.  Nodes outside 1 .. min(j0, n - 1) and padding pairs
// are zero.  Contraction is off so every value is the correctly rounded
// sequence of operations of the host's single-pair test function.
__global__ void __launch_bounds__(64) k_sweep_testfn(int n, int j0, double h, const double* __restrict__ V1r,
                                                     int npairs, int pp, const double* __restrict__ kk,
                                                     double* __restrict__ F) {
#pragma clang fp contract(off)
  constexpr int CH = 1024;                         // potential values staged per round
  __shared__ double V[CH];
  const int t = blockIdx.x * 64 + threadIdx.x;     // the grid is exactly 2 pp threads
  const int side = t / pp, c = t - side * pp;
  const bool live = c < npairs;                    // padding pairs run along and store zeros
  double* col = F + (size_t)side * (n + 1) * pp + c;
  const double k = live ? kk[side * npairs + c] : 1.0;
  const int top = j0 + 1 < n ? j0 + 1 : n;
  const double g2 = 2.0 * h * h, kh = 0.5 * k * k;
  double pm = 0.0, p0 = h;                         // phi[j-1], phi[j]
  col[0] = 0.0;
  col[(size_t)pp] = h;
  // the potential term depends on the node only: the block computes it once
  // per round, so no division sits on the recurrence's dependency chain
  for (int jc = 1; jc < top; jc += CH) {
    const int cnt = top - jc < CH ? top - jc : CH;
    __syncthreads();
    for (int i = threadIdx.x; i < cnt; i += 64) V[i] = V1r[jc + i];
    __syncthreads();
    for (int i = 0; i < cnt; ++i) {
      const double pn = (2.0 * p0 - pm) + (g2 * (V[i] - kh)) * p0;
      col[(size_t)(jc + i + 1) * pp] = pn;
      pm = p0;
      p0 = pn;
    }
  }
  const int jr = j0 < top - 1 ? j0 : top - 1;
  const double pr = sqrt(k * k - 2.0 * V1r[jr]);
  const double dphi = (col[(size_t)(jr + 1) * pp] - col[(size_t)(jr - 1) * pp]) / (2.0 * h);
  const double q = dphi / pr, f = col[(size_t)jr * pp];
  const double amp = sqrt(f * f + q * q);
  const double sc = 1.0 / (amp * sqrt(pr));
  const int last = live ? (j0 < n - 1 ? j0 : n - 1) : 0;
  // scaling pass: 16 loads in flight per group (one memory latency per group,
  // not per node), then the group's stores
  col[0] = 0.0;
  for (int jb = 1; jb <= n; jb += 16) {
    double v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) v[u] = jb + u <= last ? col[(size_t)(jb + u) * pp] : 0.0;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int j = jb + u;
      if (j <= n) col[(size_t)j * pp] = j <= last ? (j == j0 ? 0.5 * h : h) * (v[u] * sc) : 0.0;
    }
  }
}

// out[q] = sum_b part[b * 2pp + q]: SWQ quantities per block, each summed in
// 256 / SWQ slices of the blocks (enough blocks and loads in flight for the
// few hundred partials per quantity)
constexpr int SWQ = 32;
__global__ void __launch_bounds__(256) k_zeta_sweep_sum(int nb, int nq, const double* __restrict__ part,
                                                        double* __restrict__ out) {
  const int q0 = SWQ * blockIdx.x;
  const int nqb = nq - q0 < SWQ ? nq - q0 : SWQ;
  finish_sum_nt<256>(part + q0, nb, nqb, out + q0, nq);
}

// ----------------------------------------------------------------------------
// Sensitivities of the ionisation amplitude zeta (eq. double-ionization) with
// respect to p = (Z1, Z2, lambda).  With F = f2[k] f1[j] (trapezoid-weighted
// test functions on the real region) and u = A^{-1} chi:
//   d zeta/dp = sum F' (chi - V12 u) + sum F (dchi/dp - dV12/dp u)        (explicit)
//             + sum v (dchi/dp - dA/dp u),     A^T v = d zeta/du = -F V12  (adjoint)
// Adjoint right-hand side:
__global__ void __launch_bounds__(256) k_adj_rhs(int n, int pitch, int j0, const double2* __restrict__ tm,
                                                 const double* __restrict__ f1,
                                                 const double* __restrict__ f2,
                                                 double2* __restrict__ out) {
  MGC_NODE_LOOP(n, k, j) {
    v2<double> v = mk<double>(0, 0);
    if (k <= j0 && j <= j0) {
      const double w = -f2[k] * f1[j];
      v2<double> t12 = tm[j > k ? j : k];
      v = mk<double>(w * t12.x, w * t12.y);
    }
    out[(size_t)k * pitch + j] = v;
  }
}

struct TPParams { double Z1, Z2, lam, E, k0; };

// analytic d chi / d p at a real-region node (chi as built by k_rhs_tp)
__device__ __forceinline__ void dchi_dp(const TPParams& P, double xj, double xk, bool jk_max_is_j,
                                        double out[3]) {
  const double xm = jk_max_is_j ? xj : xk;
  const double pref = 2.0 * P.Z1 * sqrt(P.Z1);
  const double phj = pref * xj * exp(-P.Z1 * xj), phk = pref * xk * exp(-P.Z1 * xk);
  const double Sj = sin(P.k0 * xj), Sk = sin(P.k0 * xk);
  const double Cj = cos(P.k0 * xj), Ck = cos(P.k0 * xk);
  const double a1 = P.lam / xm - P.Z2 / xk, a2 = P.lam / xm - P.Z2 / xj;
  const double r2 = 0.70710678118654752440;
  const double dk0 = P.Z1 / P.k0;
  const double dphj = phj * (1.5 / P.Z1 - xj), dphk = phk * (1.5 / P.Z1 - xk);
  out[0] = r2 * (a1 * (dphj * Sk + phj * Ck * xk * dk0) + a2 * (dphk * Sj + phk * Cj * xj * dk0));
  out[1] = r2 * (-phj * Sk / xk - phk * Sj / xj);
  out[2] = r2 * (phj * Sk + phk * Sj) / xm;
}

// per-block partials (12 doubles): [explicit dZ1, dZ2, dlam | adjoint dZ1, dZ2, dlam], complex each
__global__ void __launch_bounds__(256) k_sens_part(int n, int pitch, int j0, const double2* __restrict__ z,
                                                   const double2* __restrict__ tm, const double* __restrict__ f1,
                                                   const double* __restrict__ f2, const double* __restrict__ df1,
                                                   const double* __restrict__ df2, const double2* __restrict__ u,
                                                   const double2* __restrict__ v, const double2* __restrict__ chi,
                                                   TPParams P, double* __restrict__ part) {
  double acc[12];
#pragma unroll
  for (int q = 0; q < 12; ++q) acc[q] = 0;
  MGC_NODE_LOOP(n, k, j) {
    const size_t idx = (size_t)k * pitch + j;
    const v2<double> uu = u[idx], vv = v[idx];
    const int mx = j > k ? j : k;
    // dA/dp u : (-u/z_j, -u/z_k, u/z_max)
    const v2<double> ij = cdiv(mk<double>(1, 0), z[j]), ik = cdiv(mk<double>(1, 0), z[k]),
                     im = cdiv(mk<double>(1, 0), z[mx]);
    v2<double> dAu[3] = {cmul(mk<double>(-ij.x, -ij.y), uu), cmul(mk<double>(-ik.x, -ik.y), uu), cmul(im, uu)};
    double dc[3] = {0, 0, 0};
    const bool real_region = (k <= j0 && j <= j0);
    if (real_region) dchi_dp(P, z[j].x, z[k].x, j > k, dc);
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      // adjoint part: v (dchi - dA u), no conjugation
      const v2<double> w = mk<double>(dc[q] - dAu[q].x, -dAu[q].y);
      const v2<double> pr = cmul(vv, w);
      acc[6 + 2 * q] += pr.x;
      acc[6 + 2 * q + 1] += pr.y;
    }
    if (real_region) {
      const double F = f2[k] * f1[j];
      const double dF = df2[k] * f1[j] + f2[k] * df1[j];
      const v2<double> src = csub(chi[idx], cmul(tm[mx], uu));
      // Z1: dF src + F dchi/dZ1 ; Z2: F dchi/dZ2 ; lambda: F (dchi/dlam - u/z_max)
      acc[0] += dF * src.x + F * dc[0];
      acc[1] += dF * src.y;
      acc[2] += F * dc[1];
      acc[4] += F * (dc[2] - dAu[2].x);
      acc[5] += F * (-dAu[2].y);
    }
  }
  double tot[12];
  block_sum<12>(acc, tot);
  if (threadIdx.x == 0)
#pragma unroll
    for (int q = 0; q < 12; ++q) part[(size_t)flat_block() * 12 + q] = tot[q];
}

// ============================================================================
// host launchers
static inline dim3 stencil_grid(int n) {
  return dim3((n - 1 + SX - 1) / SX, (n - 1 + SY * ROWS - 1) / (SY * ROWS));
}
static inline int stencil_blocks(int n) {
  dim3 g = stencil_grid(n);
  return g.x * g.y;
}
int launch_stencil_blocks(int n) { return stencil_blocks(n); }

template <typename T, typename TU, typename TF, typename TO>
void launch_stencil(hipStream_t s, const Level<T>& L, const void* u, const void* f, void* out,
                    int mode, double* part, Finish fin) {
  hipLaunchKernelGGL((k_stencil<T, TU, TF, TO>), stencil_grid(L.n), dim3(SX, SY), 0, s, L,
                     (const v2<TU>*)u, (const v2<TF>*)f, (v2<TO>*)out, mode, part);
  if (part && fin.out)
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, stencil_blocks(L.n), 2, part, fin.out,
                       fin.copy_to);
}
template void launch_stencil<double, double, double, double>(hipStream_t, const Level<double>&, const void*, const void*, void*, int, double*, Finish);
template void launch_stencil<double, float, double, double>(hipStream_t, const Level<double>&, const void*, const void*, void*, int, double*, Finish);
template void launch_stencil<float, float, float, float>(hipStream_t, const Level<float>&, const void*, const void*, void*, int, double*, Finish);

template <typename T>
void launch_jacobi(hipStream_t s, const Level<T>& L, const void* u, const void* f, void* out, double omega) {
  hipLaunchKernelGGL((k_jacobi<T>), stencil_grid(L.n), dim3(SX, SY), 0, s, L, (const v2<T>*)u,
                     (const v2<T>*)f, (v2<T>*)out, (T)omega);
}
template <typename T>
void launch_resid_restrict(hipStream_t s, const Level<T>& L, const void* u, const void* f, void* fc,
                           int pitch_c) {
  const int nc = L.n / 2;
  dim3 grid((nc - 1 + SX - 1) / SX, (nc - 1 + SY - 1) / SY);
  hipLaunchKernelGGL((k_resid_restrict<T>), grid, dim3(SX, SY), 0, s, L, (const v2<T>*)u,
                     (const v2<T>*)f, (v2<T>*)fc, pitch_c);
}
template <typename T>
void launch_prolong_add(hipStream_t s, int n, int pitch, void* u, const void* ec, int pitch_c) {
  hipLaunchKernelGGL((k_prolong_add<T>), stencil_grid(n), dim3(SX, SY), 0, s, n, pitch, (v2<T>*)u,
                     (const v2<T>*)ec, pitch_c);
}
template <typename T>
void launch_coarse_solve(hipStream_t s, const double2* Ainv, int nc, int pitch, const void* f, void* u) {
  const int N = (nc - 1) * (nc - 1);
  const int waves_per_block = 4;
  hipLaunchKernelGGL((k_coarse_solve<T>), dim3((N + waves_per_block - 1) / waves_per_block),
                     dim3(64 * waves_per_block), 0, s, Ainv, nc, pitch, (const v2<T>*)f, (v2<T>*)u);
}

template <typename T>
void launch_s1_zero(hipStream_t s, const Level<T>& L, const void* f, const double* fs, double omega,
                    void* fc, int pitch_c, bool small) {
  const int nc = L.n / 2;
  const dim3 big((nc - 1 + S1Big::CX - 1) / S1Big::CX, (nc - 1 + S1Big::CY - 1) / S1Big::CY);
  if (!small) {
    hipLaunchKernelGGL((k_s1_zero<T, S1Big>), big, dim3(64, 4), 0, s, L, (const v2<T>*)f, fs, (T)omega,
                       (v2<T>*)fc, pitch_c);
  } else {
    const dim3 sm((nc - 1 + S1Small::CX - 1) / S1Small::CX, (nc - 1 + S1Small::CY - 1) / S1Small::CY);
    hipLaunchKernelGGL((k_s1_zero<T, S1Small>), sm, dim3(64, 4), 0, s, L, (const v2<T>*)f, fs, (T)omega,
                       (v2<T>*)fc, pitch_c);
  }
}
template <typename T>
void launch_s2_zero(hipStream_t s, const Level<T>& L, const void* f, const double* fs, double omega,
                    const void* ec, int pitch_c, void* u, bool small) {
  const dim3 big((L.n - 1 + S2Big::TX - 1) / S2Big::TX, (L.n - 1 + S2Big::TY - 1) / S2Big::TY);
  if (!small) {
    hipLaunchKernelGGL((k_s2_zero<T, S2Big>), big, dim3(64, 4), 0, s, L, (const v2<T>*)f, fs, (T)omega,
                       (const v2<T>*)ec, pitch_c, (v2<T>*)u);
  } else {
    const dim3 sm((L.n - 1 + S2Small::TX - 1) / S2Small::TX, (L.n - 1 + S2Small::TY - 1) / S2Small::TY);
    hipLaunchKernelGGL((k_s2_zero<T, S2Small>), sm, dim3(64, 4), 0, s, L, (const v2<T>*)f, fs, (T)omega,
                       (const v2<T>*)ec, pitch_c, (v2<T>*)u);
  }
}

template <typename T>
void launch_tail(hipStream_t s, const TailArgs<T>& A, bool down) {
  if (down) {
    const int N = (A.nc - 1) * (A.nc - 1);
    hipLaunchKernelGGL((k_tail_down<T>), dim3((N + TROWS - 1) / TROWS), dim3(TT), 0, s, A);
  } else {
    hipLaunchKernelGGL((k_tail_up<T>), dim3((A.L[0].n - 1 + TUPR - 1) / TUPR), dim3(TT), 0, s, A);
  }
}

template <typename T>
void launch_s1_pair(hipStream_t s, const Level<T>& Lf, const Level<T>& Lc, const void* f, const double* fs,
                    double omega, void* f1, int pitch1, void* f2, int pitch2) {
  const int n2 = Lc.n / 2;
  const dim3 grid((n2 - 1 + S1Small::CX - 1) / S1Small::CX, (n2 - 1 + S1Small::CY - 1) / S1Small::CY);
  hipLaunchKernelGGL((k_s1_pair<T>), grid, dim3(64, 16), 0, s, Lf, Lc, (const v2<T>*)f, fs, (T)omega,
                     (v2<T>*)f1, pitch1, (v2<T>*)f2, pitch2);
}
template <typename T>
void launch_s2_pair(hipStream_t s, const Level<T>& Lf, const Level<T>& Lc, const void* f, const double* fs,
                    double omega, const void* fc, const void* ecc, int pitch_cc, void* u) {
  const dim3 grid((Lf.n - 1 + S2Small::TX - 1) / S2Small::TX, (Lf.n - 1 + S2Small::TY - 1) / S2Small::TY);
  hipLaunchKernelGGL((k_s2_pair<T>), grid, dim3(64, 4), 0, s, Lf, Lc, (const v2<T>*)f, fs,
                     (const v2<T>*)fc, (const v2<T>*)ecc, pitch_cc, (T)omega, (v2<T>*)u);
}

#define MGC_INST_LEVEL(T)                                                                      \
  template void launch_jacobi<T>(hipStream_t, const Level<T>&, const void*, const void*, void*, double); \
  template void launch_resid_restrict<T>(hipStream_t, const Level<T>&, const void*, const void*, void*, int); \
  template void launch_prolong_add<T>(hipStream_t, int, int, void*, const void*, int);        \
  template void launch_coarse_solve<T>(hipStream_t, const double2*, int, int, const void*, void*); \
  template void launch_s1_zero<T>(hipStream_t, const Level<T>&, const void*, const double*, double, void*, int, \
                                  bool);                                                                      \
  template void launch_s2_zero<T>(hipStream_t, const Level<T>&, const void*, const double*, double, const void*, \
                                  int, void*, bool);                                                          \
  template void launch_tail<T>(hipStream_t, const TailArgs<T>&, bool);                        \
  template void launch_s2_pair<T>(hipStream_t, const Level<T>&, const Level<T>&, const void*, const double*, \
                                  double, const void*, const void*, int, void*);                 \
  template void launch_s1_pair<T>(hipStream_t, const Level<T>&, const Level<T>&, const void*, const double*, \
                                  double, void*, int, void*, int);
MGC_INST_LEVEL(double)
MGC_INST_LEVEL(float)

template <typename T>
void launch_cccs(hipStream_t s, const Level<T>& L, void* u, const void* f, const double* fs,
                 const ChanTab<T>& ch, const ChanSys<T>& SA, const ChanSys<T>& SB,
                 const CccsScratch& w, const MarkHook* hook) {
  auto mark = [&](int kind, int end) {
    if (hook && hook->fn && hook->kind == kind) hook->fn(hook->ctx, s, end);
  };
  const int n = L.n;
  const int MC = ch.M > ch.L ? ch.M : ch.L;
  v2<T>* partA = (v2<T>*)w.partA;
  v2<T>* partB = (v2<T>*)w.partB;
  v2<T>* rhoA = (v2<T>*)w.rhoA;
  v2<T>* rhoB = (v2<T>*)w.rhoB;
  v2<T>* partC = (v2<T>*)w.partC;
  v2<T>* gA = (v2<T>*)w.gA;
  v2<T>* gB = (v2<T>*)w.gB;
  v2<T>* YA = (v2<T>*)w.YA;
  v2<T>* YB = (v2<T>*)w.YB;
  v2<T>* eA = (v2<T>*)w.eA;
  v2<T>* eB = (v2<T>*)w.eB;
  const int nt = (n - 1 + PT - 1) / PT;
#define MGC_CC_DISPATCH(KERNEL, GRID, BLOCK, ...)                                      \
  if (MC <= 4) hipLaunchKernelGGL((KERNEL<T, 4>), GRID, BLOCK, 0, s, __VA_ARGS__);      \
  else if (MC <= 8) hipLaunchKernelGGL((KERNEL<T, 8>), GRID, BLOCK, 0, s, __VA_ARGS__); \
  else hipLaunchKernelGGL((KERNEL<T, 16>), GRID, BLOCK, 0, s, __VA_ARGS__);
  mark(1, 0);
#define MGC_PROJ(MCC)                                                                               \
  hipLaunchKernelGGL((k_cccs_project<T, MCC>), dim3(nt, nt), dim3(64, ProjCfg<T, MCC>::W), 0, s, L,   \
                     (const v2<T>*)u, (const v2<T>*)f, fs, ch, partA, partB)
  if (MC <= 4) {
    MGC_PROJ(4);
  } else if (MC <= 8) {
    MGC_PROJ(8);
  } else {
    MGC_PROJ(16);
  }
#undef MGC_PROJ
  mark(1, 1);
  const int nrb = launch_cccs_reduce_blocks(n);
  hipLaunchKernelGGL((k_cccs_reduce<T>), dim3(nrb), dim3(RT), 0, s, n, nt, ch, (const v2<T>*)partA,
                     (const v2<T>*)partB, rhoA, rhoB, partC);
  const int P = SA.P > SB.P ? SA.P : SB.P;
  // entries per lane: chains over M x M blocks, interface over 2M x 2M blocks
  // dynamic LDS: one chunk (chains) or all interfaces (interface sweeps)
  const int NN = SA.N > SB.N ? SA.N : SB.N;
  const int PP = SA.P < SB.P ? SA.P : SB.P;
  const int maxlen = (NN + PP - 1) / PP;
  const int Qmax = P - 1;
#define MGC_CHAIN(MCC)                                                                                 \
  mark(2, 0);                                                                                          \
  hipLaunchKernelGGL((k_cccs_chain<T, MCC>), dim3(P, 2), dim3(64),                                     \
                     (size_t)maxlen * (MCC + 2) * sizeof(v2<T>), s, SA, SB, ch, n, (const v2<T>*)rhoA,   \
                     (const v2<T>*)rhoB, (const v2<T>*)partC, nrb, gA, gB, (v2<T>*)w.HA, (v2<T>*)w.HB,   \
                     maxlen);                                                                           \
  mark(2, 1);                                                                                          \
  if (Qmax > 0)                                                                                        \
    hipLaunchKernelGGL((k_cccs_iface_mv<T>), dim3((Qmax * 2 * MC + 3) / 4, 2), dim3(256), 0, s, SA, SB,  \
                       YA, YB, (const v2<T>*)w.HA, (const v2<T>*)w.HB)
  if (MC <= 4) {
    MGC_CHAIN(4);
  } else if (MC <= 8) {
    MGC_CHAIN(8);
  } else {
    MGC_CHAIN(16);
  }
#undef MGC_CHAIN
  const int NM = (SA.N * SA.M > SB.N * SB.M) ? SA.N * SA.M : SB.N * SB.M;
#define MGC_RETRIEVE(MCC)                                                                              \
  hipLaunchKernelGGL((k_cccs_retrieve<T, MCC>), dim3((NM + 63) / 64, 2), dim3(64), 0, s, SA, SB,        \
                     (const v2<T>*)gA, (const v2<T>*)gB, (const v2<T>*)YA, (const v2<T>*)YB, eA, eB)
  if (MC <= 4) {
    MGC_RETRIEVE(4);
  } else if (MC <= 8) {
    MGC_RETRIEVE(8);
  } else {
    MGC_RETRIEVE(16);
  }
#undef MGC_RETRIEVE
  mark(3, 0);
  MGC_CC_DISPATCH(k_cccs_expand, stencil_grid(n), dim3(SX, SY), n, L.pitch, (v2<T>*)u, ch,
                  (const v2<T>*)eA, (const v2<T>*)eB);
  mark(3, 1);
#undef MGC_CC_DISPATCH
}
template void launch_cccs<double>(hipStream_t, const Level<double>&, void*, const void*, const double*,
                                  const ChanTab<double>&, const ChanSys<double>&, const ChanSys<double>&,
                                  const CccsScratch&, const MarkHook*);
template void launch_cccs<float>(hipStream_t, const Level<float>&, void*, const void*, const double*,
                                 const ChanTab<float>&, const ChanSys<float>&, const ChanSys<float>&,
                                 const CccsScratch&, const MarkHook*);

static inline dim3 vec_grid(int n) {
  const int gx = (n - 1 + 63) / 64;
  int gy = VEC_BLOCKS / gx;
  const int rows4 = (n - 1 + 3) / 4;
  if (gy > rows4) gy = rows4;
  if (gy < 1) gy = 1;
  return dim3(gx, gy);
}
static inline int vec_blocks(int n) {
  dim3 g = vec_grid(n);
  return g.x * g.y;
}
int launch_vec_blocks(int n) { return vec_blocks(n); }

// k_apply_dot grid: 64-column tiles in x, at most AX_BLOCKS blocks in all;
// every thread walks `rows` consecutive rows.
struct ApplyGrid { dim3 grid; int rows; };
static inline ApplyGrid apply_dot_grid(int n) {
  const int gx = (n - 1 + SX - 1) / SX;
  int gy = (n - 1 + AD_SY * 8 - 1) / (AD_SY * 8);
  const int cap = AX_BLOCKS / gx > 1 ? AX_BLOCKS / gx : 1;
  if (gy > cap) gy = cap;
  const int rows = (n - 1 + gy * AD_SY - 1) / (gy * AD_SY);
  return {dim3(gx, gy), rows};
}
static inline int axpy_blocks(int n, int pitch) {
  const size_t Nf = (size_t)(n + 1) * pitch;
  size_t b = (Nf + (size_t)AB * 4 - 1) / ((size_t)AB * 4);
  return (int)(b < 1 ? 1 : (b > AX_BLOCKS ? AX_BLOCKS : b));
}

// one instantiation per basis size J = 1 .. 16 (the library caps the restart
// length at 16); other J launch nothing
#define MGC_JSWITCH(M)                                                                      \
  switch (J) {                                                                              \
    case 1: M(1); break;   case 2: M(2); break;   case 3: M(3); break;   case 4: M(4); break; \
    case 5: M(5); break;   case 6: M(6); break;   case 7: M(7); break;   case 8: M(8); break; \
    case 9: M(9); break;   case 10: M(10); break; case 11: M(11); break; case 12: M(12); break; \
    case 13: M(13); break; case 14: M(14); break; case 15: M(15); break; case 16: M(16); break; \
    default: break;                                                                         \
  }

template <typename TZ>
void launch_apply_dot(hipStream_t s, const Level<double>& L, const void* z, size_t stride,
                      const double2* W, int J, double2* Y, double* part0) {
  const ApplyGrid ag = apply_dot_grid(L.n);
#define MGC_AD(JT)                                                                               \
  hipLaunchKernelGGL((k_apply_dot<TZ, JT>), ag.grid, dim3(SX, AD_SY), 0, s, L, (const v2<TZ>*)z, W, \
                     stride, Y, part0, ag.rows)
  MGC_JSWITCH(MGC_AD)
#undef MGC_AD
}
template void launch_apply_dot<double>(hipStream_t, const Level<double>&, const void*, size_t, const double2*,
                                       int, double2*, double*);
template void launch_apply_dot<float>(hipStream_t, const Level<double>&, const void*, size_t, const double2*,
                                      int, double2*, double*);

void launch_axpy_pass(hipStream_t s, int n, int pitch, size_t stride, const double2* W, int J,
                      double2* Y, float2* Y32, const double* part0, double* part1, const GmresState& st) {
  const size_t Nf = (size_t)(n + 1) * pitch;
  const int nb = axpy_blocks(n, pitch);
  const int nb0 = (int)(apply_dot_grid(n).grid.x * apply_dot_grid(n).grid.y);
#define MGC_AXD(JT)                                                                                 \
  hipLaunchKernelGGL((k_axpy_pass<JT>), dim3(nb), dim3(AB), 0, s, Nf, stride, W, Y, Y32, part0, nb0, part1, st)
  MGC_JSWITCH(MGC_AXD)
#undef MGC_AXD
}

void launch_reorth_step(hipStream_t s, int n, int pitch, size_t stride, const double2* W, int J, double2* Y,
                        float2* Y32, const double* part0, const double* part1, double* part2, const GmresState& st, int m,
                        int mm, double tol_abs, double eta) {
  const size_t Nf = (size_t)(n + 1) * pitch;
  const int nb = axpy_blocks(n, pitch);
  const int nb0 = (int)(apply_dot_grid(n).grid.x * apply_dot_grid(n).grid.y);
  const int j = J - 1;
#define MGC_RS(JT)                                                                                  \
  hipLaunchKernelGGL((k_reorth_step<JT>), dim3(nb), dim3(AB), 0, s, Nf, stride, W, Y, Y32, part1, nb, part2, st, \
                     part0, nb0, j, m, mm, tol_abs, eta)
  MGC_JSWITCH(MGC_RS)
#undef MGC_RS
}
#undef MGC_JSWITCH
template <typename TZ>
void launch_update(hipStream_t s, int n, int pitch, size_t stride, const void* Z, int J,
                   const double2* coef, double2* u) {
  hipLaunchKernelGGL((k_update<TZ, 32>), vec_grid(n), dim3(256), 0, s, n, pitch, stride,
                     (const v2<TZ>*)Z, J, coef, u);
}
template void launch_update<double>(hipStream_t, int, int, size_t, const void*, int, const double2*, double2*);
template void launch_update<float>(hipStream_t, int, int, size_t, const void*, int, const double2*, double2*);

template <typename TI, typename TO>
void launch_scale_copy(hipStream_t s, int n, int pitch_in, int pitch_out, const void* in,
                       const double* sc, void* out) {
  hipLaunchKernelGGL((k_scale_copy<TI, TO>), vec_grid(n), dim3(256), 0, s, n, pitch_in,
                     pitch_out, (const v2<TI>*)in, sc, (v2<TO>*)out);
}
template void launch_scale_copy<double, double>(hipStream_t, int, int, int, const void*, const double*, void*);
template void launch_scale_copy<double, float>(hipStream_t, int, int, int, const void*, const double*, void*);
template void launch_scale_copy<float, double>(hipStream_t, int, int, int, const void*, const double*, void*);
template void launch_scale_copy<float, float>(hipStream_t, int, int, int, const void*, const double*, void*);

void launch_weight(hipStream_t s, int n, int pitch, const double2* w, int divide, const double2* in,
                   double2* out) {
  hipLaunchKernelGGL(k_weight, vec_grid(n), dim3(256), 0, s, n, pitch, w, divide, in, out);
}
void launch_sum_partials(hipStream_t s, int nb, int nq, const double* part, double* out) {
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, nb, nq, part, out, (double*)nullptr);
}
void launch_gmres_begin(hipStream_t s, const GmresState& st, int m) {
  hipLaunchKernelGGL(k_gmres_begin, dim3(1), dim3(1), 0, s, st, m);
}
void launch_ir_scale(hipStream_t s, const double* nrm2, double Nn, double* sc) {
  hipLaunchKernelGGL(k_ir_scale, dim3(1), dim3(1), 0, s, nrm2, Nn, sc);
}
void launch_cycle_end(hipStream_t s, int n, const double* part, double* scal, const GmresState& st, int m,
                      double* rep) {
  hipLaunchKernelGGL(k_cycle_end, dim3(1), dim3(256), 0, s, stencil_blocks(n), part, scal, st, m, rep);
}
void launch_copy_scalar(hipStream_t s, const double* src, double* dst) {
  hipLaunchKernelGGL(k_copy_scalar, dim3(1), dim3(1), 0, s, src, dst);
}
void launch_fill_zero(hipStream_t s, void* p, size_t bytes) {
  hipLaunchKernelGGL(k_fill_zero, dim3(256), dim3(256), 0, s, bytes / 16, (double2*)p);
}
void launch_rhs_tp(hipStream_t s, int n, int pitch, int j0, const double2* z, double Z1, double Z2,
                   double lam, double k0, double2* chi) {
  hipLaunchKernelGGL(k_rhs_tp, vec_grid(n), dim3(256), 0, s, n, pitch, j0, z, Z1, Z2, lam, k0, chi);
}
void launch_adj_rhs(hipStream_t s, int n, int pitch, int j0, const double2* tm, const double* f1,
                    const double* f2, double2* out) {
  hipLaunchKernelGGL(k_adj_rhs, vec_grid(n), dim3(256), 0, s, n, pitch, j0, tm, f1, f2, out);
}
void launch_sens_part(hipStream_t s, int n, int pitch, int j0, const double2* z, const double2* tm,
                      const double* f1, const double* f2, const double* df1, const double* df2,
                      const double2* u, const double2* v, const double2* chi, double Z1, double Z2,
                      double lam, double E, double* part) {
  TPParams P{Z1, Z2, lam, E, sqrt(2.0 * E + Z1 * Z1)};
  hipLaunchKernelGGL(k_sens_part, vec_grid(n), dim3(256), 0, s, n, pitch, j0, z, tm, f1, f2, df1, df2,
                     u, v, chi, P, part);
}
void launch_zeta_part(hipStream_t s, int n, int pitch, int j0, const double2* tm, const double* f1,
                      const double* f2, const double2* u, const double2* chi, double* part) {
  hipLaunchKernelGGL(k_zeta_part, vec_grid(n), dim3(256), 0, s, n, pitch, j0, tm, f1, f2, u, chi, part);
}
int zeta_sweep_blocks(int top) { return ((top + SWR - 1) / SWR) * SWJ; }
void launch_sweep_testfn(hipStream_t s, int n, int j0, double h, const double* V1r, int npairs, int pp,
                         const double* kk, double* F) {
  hipLaunchKernelGGL(k_sweep_testfn, dim3((2 * pp + 63) / 64), dim3(64), 0, s, n, j0, h, V1r, npairs, pp, kk, F);
}

// s = chi - V12 u with a general two-body table (the source of the amplitude
// integrals under a potential model without the lambda / z_max form)
__global__ void __launch_bounds__(256) k_src_v12(int n, int pitch, const double2* __restrict__ chi,
                                                 const double2* __restrict__ v12, const double2* __restrict__ u,
                                                 double2* __restrict__ out) {
  MGC_NODE_LOOP(n, k, j) {
    const size_t idx = (size_t)k * pitch + j;
    out[idx] = csub(chi[idx], cmul(v12[idx], u[idx]));
  }
}
void launch_src_v12(hipStream_t s, int n, int pitch, const double2* chi, const double2* v12, const double2* u,
                    double2* out) {
  hipLaunchKernelGGL(k_src_v12, vec_grid(n), dim3(256), 0, s, n, pitch, chi, v12, u, out);
}
// ----------------------------------------------------------------------------
// GMRES(3) smoothing substitute of the V-cycle (Sec. 6.1), on one level:
// u += V y with y minimising ||f - A(u + V y)|| over K_3(A, r0):
//   V0 = f - A u (k_stencil, ||V0||^2 partials);  V0 /= beta   k_gs_normalize
//   for i = 0, 1, 2:  V_{i+1} = A V_i, V_q^H V_{i+1}         k_gs_arnoldi
//                     H[q][i] = V_q^H V_{i+1}, V_{i+1} -= sum H[q][i] V_q,
//                     ||V_{i+1}||^2                           k_gs_orth
//                     H[i+1][i] = ||V_{i+1}||, V_{i+1} /= it  k_gs_normalize
//   y = argmin ||beta e1 - H y|| by Givens rotations         k_gs_solve
//   u += sum y_i V_i                                         k_gs_update
// Classical Gram-Schmidt in one pass; an exact breakdown (a zero norm) ends
// the space there.  State st (doubles): H (4 x 3 complex, column-major) at 0,
// beta at GS_BETA, y (3 complex) at GS_Y.
constexpr int GS_M = 3, GS_BETA = 24, GS_Y = 26;
__device__ __forceinline__ int gs_h(int row, int col) { return 2 * (col * (GS_M + 1) + row); }

template <typename T>
__global__ void __launch_bounds__(256) k_gs_normalize(int n, int pitch, v2<T>* __restrict__ V,
                                                      const double* __restrict__ part, int nb, int pstride,
                                                      double* __restrict__ st, int slot) {
  __shared__ double nn[1];
  finish_sum_nt<256>(part, nb, 1, nn, pstride);
  const double nrm = sqrt(nn[0]);
  if (flat_block() == 0 && threadIdx.x == 0) {
    st[slot] = nrm;
    if (slot != GS_BETA) st[slot + 1] = 0.0;
  }
  const T sc = nrm > 0.0 ? (T)(1.0 / nrm) : T(0);
  MGC_NODE_LOOP(n, k, j) {
    const size_t idx = (size_t)k * pitch + j;
    V[idx] = cscale(V[idx], sc);
  }
}
template <typename T, int J>
__global__ void __launch_bounds__(256) k_gs_arnoldi(Level<T> L, v2<T>* __restrict__ V, size_t stride,
                                                    double* __restrict__ part) {
  double acc[2 * J];
#pragma unroll
  for (int q = 0; q < 2 * J; ++q) acc[q] = 0.0;
  const int n = L.n, p = L.pitch;
  MGC_NODE_LOOP(n, k, j) {
    const size_t idx = (size_t)k * p + j;
    const v2<T> w = apply_at<T>(L, V + (size_t)(J - 1) * stride, k, j);
    V[(size_t)J * stride + idx] = w;
#pragma unroll
    for (int q = 0; q < J; ++q) {
      const v2<T> v = V[(size_t)q * stride + idx];
      acc[2 * q] += (double)v.x * w.x + (double)v.y * w.y;
      acc[2 * q + 1] += (double)v.x * w.y - (double)v.y * w.x;
    }
  }
  double tot[2 * J];
  block_sum<2 * J>(acc, tot);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < 2 * J; ++q) part[(size_t)flat_block() * (2 * J) + q] = tot[q];
  }
}
template <typename T, int J>
__global__ void __launch_bounds__(256) k_gs_orth(int n, int pitch, v2<T>* __restrict__ V, size_t stride,
                                                 const double* __restrict__ pin, int nbin, double* __restrict__ st,
                                                 double* __restrict__ pout) {
  __shared__ double h[2 * J];
  finish_sum_nt<256>(pin, nbin, 2 * J, h);
  if (flat_block() == 0 && threadIdx.x < 2 * J) st[gs_h(threadIdx.x / 2, J - 1) + (threadIdx.x & 1)] = h[threadIdx.x];
  v2<T> c[J];
#pragma unroll
  for (int q = 0; q < J; ++q) c[q] = mk<T>((T)h[2 * q], (T)h[2 * q + 1]);
  double acc[1] = {0.0};
  MGC_NODE_LOOP(n, k, j) {
    const size_t idx = (size_t)k * pitch + j;
    v2<T> w = V[(size_t)J * stride + idx];
#pragma unroll
    for (int q = 0; q < J; ++q) w = csub(w, cmul(c[q], V[(size_t)q * stride + idx]));
    V[(size_t)J * stride + idx] = w;
    acc[0] += (double)w.x * w.x + (double)w.y * w.y;
  }
  double tot[1];
  block_sum<1>(acc, tot);
  if (threadIdx.x == 0) pout[flat_block()] = tot[0];
}
__global__ void k_gs_solve(double* st) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double2 H[GS_M + 1][GS_M], g[GS_M + 1];
  for (int c = 0; c < GS_M; ++c)
    for (int r = 0; r <= GS_M; ++r) H[r][c] = make_double2(st[gs_h(r, c)], st[gs_h(r, c) + 1]);
  for (int r = 0; r <= GS_M; ++r) g[r] = make_double2(0.0, 0.0);
  g[0] = make_double2(st[GS_BETA], 0.0);
  int kd = GS_M;
  for (int i = 0; i < GS_M; ++i)
    if (H[i + 1][i].x == 0.0 && H[i + 1][i].y == 0.0) { kd = i + 1; break; }
  double2 y[GS_M];
  for (int i = 0; i < GS_M; ++i) y[i] = make_double2(0.0, 0.0);
  if (st[GS_BETA] > 0.0) {
    // Givens rotations G_i = [conj(c) conj(s); -s c] zero H[i+1][i]
    for (int i = 0; i < kd; ++i) {
      const double2 a = H[i][i], b = H[i + 1][i];
      const double den = sqrt(a.x * a.x + a.y * a.y + b.x * b.x + b.y * b.y);
      const double2 c = make_double2(a.x / den, a.y / den), sn = make_double2(b.x / den, b.y / den);
      for (int col = i; col < kd; ++col) {
        const double2 x1 = H[i][col], x2 = H[i + 1][col];
        H[i][col] = cadd(cmul(make_double2(c.x, -c.y), x1), cmul(make_double2(sn.x, -sn.y), x2));
        H[i + 1][col] = csub(cmul(c, x2), cmul(sn, x1));
      }
      const double2 g1 = g[i], g2 = g[i + 1];
      g[i] = cadd(cmul(make_double2(c.x, -c.y), g1), cmul(make_double2(sn.x, -sn.y), g2));
      g[i + 1] = csub(cmul(c, g2), cmul(sn, g1));
    }
    for (int i = kd - 1; i >= 0; --i) {
      double2 acc = g[i];
      for (int c = i + 1; c < kd; ++c) acc = csub(acc, cmul(H[i][c], y[c]));
      y[i] = cdiv(acc, H[i][i]);
    }
  }
  for (int i = 0; i < GS_M; ++i) {
    st[GS_Y + 2 * i] = y[i].x;
    st[GS_Y + 2 * i + 1] = y[i].y;
  }
}
template <typename T>
__global__ void __launch_bounds__(256) k_gs_update(int n, int pitch, const v2<T>* __restrict__ V, size_t stride,
                                                   const double* __restrict__ st, v2<T>* __restrict__ u) {
  v2<T> y[GS_M];
#pragma unroll
  for (int q = 0; q < GS_M; ++q) y[q] = mk<T>((T)st[GS_Y + 2 * q], (T)st[GS_Y + 2 * q + 1]);
  MGC_NODE_LOOP(n, k, j) {
    const size_t idx = (size_t)k * pitch + j;
    v2<T> v = u[idx];
#pragma unroll
    for (int q = 0; q < GS_M; ++q) v = cadd(v, cmul(y[q], V[(size_t)q * stride + idx]));
    u[idx] = v;
  }
}

// ----------------------------------------------------------------------------
// GMRES(3)-smoothed coarse tail in one workgroup (512 threads): every level
// from the top one (n <= GT_MAX_N) down to the coarsest.  The smoothing
// vectors of a level live in registers (NP nodes per thread, node index
// tid + 512 q in row-major interior order); the vector the operator is
// applied to is written to one LDS tile X (stride GT_W, zero ring), the 1D
// tables of the level to LDS.  Block-wide sums: wave sums, then the 8 wave
// partials in a fixed order (deterministic).  Per level and step the
// arithmetic is that of k_gs_* (classical Gram-Schmidt in one pass, norms of
// the orthogonalised vectors, Givens least squares), k_resid_restrict,
// k_coarse_solve and k_prolong_add; only the order of the dot-product sums
// differs.
constexpr int GT_THREADS = 512, GT_WAVES = GT_THREADS / 64, GT_W = GT_MAX_N + 1, GT_NR = 8;

template <int NV>
__device__ __forceinline__ void gt_reduce(double (&v)[NV], double* red) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] = wave_sum(v[q]);
  __syncthreads();                               // the previous sum's readers are done
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) red[w * GT_NR + q] = v[q];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    double t = 0.0;
    for (int i = 0; i < GT_WAVES; ++i) t += red[i * GT_NR + q];
    v[q] = t;
  }
}

// stage the 1D tables of level L and zero the ring of an n-level tile in X
template <typename T>
__device__ __forceinline__ void gt_level_setup(const Level<T>& L, v2<T>* X, v2<T> (*tb)[GT_W]) {
  const int n = L.n, tid = threadIdx.x;
  __syncthreads();                               // X and the tables are free
  for (int i = tid; i <= n; i += GT_THREADS) {
    const bool in = i > 0 && i < n;
    tb[0][i] = in ? L.a[i] : mk<T>(0, 0);
    tb[1][i] = in ? L.c[i] : mk<T>(0, 0);
    tb[2][i] = in ? L.px[i] : mk<T>(0, 0);
    tb[3][i] = in ? L.py[i] : mk<T>(0, 0);
    tb[4][i] = in ? L.tm[i] : mk<T>(0, 0);
  }
  for (int i = tid; i < 4 * (n + 1); i += GT_THREADS) {
    const int side = i / (n + 1), t = i % (n + 1);
    const int k = side == 0 ? 0 : (side == 1 ? n : t), j = side == 0 || side == 1 ? t : (side == 2 ? 0 : n);
    X[k * GT_W + j] = mk<T>(0, 0);
  }
}

// (A x)(k, j) with x in the tile X (the arithmetic of apply_at)
template <typename T>
__device__ __forceinline__ v2<T> gt_apply(const Level<T>& L, const v2<T>* X, const v2<T> (*tb)[GT_W], int k, int j) {
  v2<T> d = cadd(cadd(tb[2][j], tb[3][k]), tb[4][j > k ? j : k]);
  if (L.v12) d = cadd(d, v12_at(L, k, j));
  d.x -= L.E;
  v2<T> acc = cmul(d, X[k * GT_W + j]);
  acc = cfma(acc, tb[0][j], X[k * GT_W + j - 1]);
  acc = cfma(acc, tb[1][j], X[k * GT_W + j + 1]);
  acc = cfma(acc, tb[0][k], X[(k - 1) * GT_W + j]);
  acc = cfma(acc, tb[1][k], X[(k + 1) * GT_W + j]);
  return acc;
}

// node q of this thread on a level with m = n - 1 interior points per row
__device__ __forceinline__ bool gt_node(int q, int m, int& k, int& j) {
  const int idx = threadIdx.x + GT_THREADS * q;
  if (idx >= m * m) return false;
  k = idx / m + 1;
  j = idx - (k - 1) * m + 1;
  return true;
}

template <typename T, int NP>
__device__ __forceinline__ void gt_store(v2<T>* X, const v2<T> (&x)[NP], int m) {
  __syncthreads();                               // the tile's readers are done
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    int k, j;
    if (gt_node(q, m, k, j)) X[k * GT_W + j] = x[q];
  }
  __syncthreads();
}

// Least squares min ||beta e1 - H y|| by Givens rotations on the k x k+1
// Hessenberg matrix (the arithmetic of k_gs_solve); H destroyed.
__device__ void gt_lsq(double2 (*H)[GS_M], double beta, int kd, double2* y) {
  double2 g[GS_M + 1];
  for (int r = 0; r <= GS_M; ++r) g[r] = make_double2(0.0, 0.0);
  g[0] = make_double2(beta, 0.0);
  for (int i = 0; i < kd; ++i) {
    const double2 a = H[i][i], b = H[i + 1][i];
    const double den = sqrt(a.x * a.x + a.y * a.y + b.x * b.x + b.y * b.y);
    const double2 c = make_double2(a.x / den, a.y / den), sn = make_double2(b.x / den, b.y / den);
    for (int col = i; col < kd; ++col) {
      const double2 x1 = H[i][col], x2 = H[i + 1][col];
      H[i][col] = cadd(cmul(make_double2(c.x, -c.y), x1), cmul(make_double2(sn.x, -sn.y), x2));
      H[i + 1][col] = csub(cmul(c, x2), cmul(sn, x1));
    }
    const double2 g1 = g[i], g2 = g[i + 1];
    g[i] = cadd(cmul(make_double2(c.x, -c.y), g1), cmul(make_double2(sn.x, -sn.y), g2));
    g[i + 1] = csub(cmul(c, g2), cmul(sn, g1));
  }
  for (int i = 0; i < GS_M; ++i) y[i] = make_double2(0.0, 0.0);
  for (int i = kd - 1; i >= 0; --i) {
    double2 acc = g[i];
    for (int c = i + 1; c < kd; ++c) acc = csub(acc, cmul(H[i][c], y[c]));
    y[i] = cdiv(acc, H[i][i]);
  }
}

// One GMRES(3) smoothing step on level L, in place on u (global, pitch pu):
// u += V y.  The basis V lives in registers; the operator is applied to the
// tile X, and A V_j is formed twice (once for the projections, once for the
// orthogonalised vector) rather than kept, to save registers.  The
// Hessenberg matrix and y live in LDS, the least squares is solved by one
// thread.
template <typename T, int NP>
__device__ void gt_gmres3(const Level<T>& L, v2<T>* X, const v2<T> (*tb)[GT_W], double* red, double2 (*H)[GS_M],
                          double2* ys, v2<T>* __restrict__ u, int pu, const v2<T>* __restrict__ f, int pf) {
  const int m = L.n - 1;
  v2<T> V[GS_M][NP];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    int k, j;
    if (gt_node(q, m, k, j)) X[k * GT_W + j] = u[(size_t)k * pu + j];
  }
  __syncthreads();
  double nn[1] = {0.0};
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    int k, j;
#pragma unroll
    for (int i = 0; i < GS_M; ++i) V[i][q] = mk<T>(0, 0);
    if (gt_node(q, m, k, j)) {
      const v2<T> r = csub(f[(size_t)k * pf + j], gt_apply(L, X, tb, k, j));
      V[0][q] = r;
      nn[0] += (double)r.x * r.x + (double)r.y * r.y;
    }
  }
  gt_reduce<1>(nn, red);
  const double beta = sqrt(nn[0]);
  if (!(beta > 0.0)) return;
  {
    const T sc = (T)(1.0 / beta);
#pragma unroll
    for (int q = 0; q < NP; ++q) V[0][q] = cscale(V[0][q], sc);
  }
  int kd = GS_M;
#pragma unroll
  for (int jj = 0; jj < GS_M; ++jj) {
    gt_store<T, NP>(X, V[jj], m);
    double hd[2 * GS_M];
#pragma unroll
    for (int t = 0; t < 2 * GS_M; ++t) hd[t] = 0.0;
#pragma unroll
    for (int q = 0; q < NP; ++q) {
      int k, j;
      if (gt_node(q, m, k, j)) {
        const v2<T> w = gt_apply(L, X, tb, k, j);
#pragma unroll
        for (int i = 0; i <= jj; ++i) {
          const v2<T> v = V[i][q];
          hd[2 * i] += (double)v.x * w.x + (double)v.y * w.y;
          hd[2 * i + 1] += (double)v.x * w.y - (double)v.y * w.x;
        }
      }
    }
    gt_reduce<2 * GS_M>(hd, red);
    double n2[1] = {0.0};
#pragma unroll
    for (int q = 0; q < NP; ++q) {
      int k, j;
      if (gt_node(q, m, k, j)) {
        v2<T> w = gt_apply(L, X, tb, k, j);
#pragma unroll
        for (int i = 0; i <= jj; ++i) w = csub(w, cmul(mk<T>((T)hd[2 * i], (T)hd[2 * i + 1]), V[i][q]));
        n2[0] += (double)w.x * w.x + (double)w.y * w.y;
        if (jj + 1 < GS_M) V[jj + 1][q] = w;
      }
    }
    gt_reduce<1>(n2, red);
    const double hn = sqrt(n2[0]);
    if (threadIdx.x == 0) {
#pragma unroll
      for (int i = 0; i <= GS_M; ++i) H[i][jj] = make_double2(i <= jj ? hd[2 * i] : 0.0, i <= jj ? hd[2 * i + 1] : 0.0);
      H[jj + 1][jj] = make_double2(hn, 0.0);
    }
    if (hn == 0.0) {
      kd = jj + 1;
      break;
    }
    if (jj + 1 < GS_M) {
      const T sc = (T)(1.0 / hn);
#pragma unroll
      for (int q = 0; q < NP; ++q) V[jj + 1][q] = cscale(V[jj + 1][q], sc);
    }
  }
  if (threadIdx.x == 0) gt_lsq(H, beta, kd, ys);
  __syncthreads();
  v2<T> yv[GS_M];
#pragma unroll
  for (int i = 0; i < GS_M; ++i) yv[i] = mk<T>((T)ys[i].x, (T)ys[i].y);
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    int k, j;
    if (gt_node(q, m, k, j)) {
      v2<T> uv = u[(size_t)k * pu + j];
#pragma unroll
      for (int i = 0; i < GS_M; ++i)
        if (i < kd) uv = cadd(uv, cmul(yv[i], V[i][q]));
      u[(size_t)k * pu + j] = uv;
    }
  }
}

// member i of a kernel-argument array with a uniform runtime index, by
// selects (no dynamic indexing, which would copy the arguments to scratch)
template <typename X>
__device__ __forceinline__ X gt_pick(const X (&a)[TMAXL], int i) {
  static_assert(TMAXL == 4, "gt_pick covers four entries");
  return i == 0 ? a[0] : (i == 1 ? a[1] : (i == 2 ? a[2] : a[3]));
}
template <typename X>
__device__ __forceinline__ X gt_pick1(const X (&a)[TMAXL + 1], int i) {
  static_assert(TMAXL == 4, "gt_pick1 covers five entries");
  return i == 0 ? a[0] : (i == 1 ? a[1] : (i == 2 ? a[2] : (i == 3 ? a[3] : a[4])));
}

template <typename T, int NP>
__global__ void __launch_bounds__(GT_THREADS) k_gs_tail(GsTailArgs<T> A) {
  __shared__ v2<T> X[GT_W * GT_W];
  __shared__ v2<T> tb[5][GT_W];
  __shared__ double red[GT_WAVES * GT_NR];
  __shared__ double2 H[GS_M + 1][GS_M];
  __shared__ double2 ys[GS_M];
  const int tid = threadIdx.x;
  // down: pre-smoothing (iterate in its level's field), residual,
  // full-weighting restriction
  for (int i = 0; i < A.nl; ++i) {
    const Level<T> L = gt_pick(A.L, i);
    const int n = L.n, m = n - 1;
    const v2<T>* f = i == 0 ? A.f0 : gt_pick1(A.f, i);
    const int pf = i == 0 ? L.pitch : gt_pick1(A.pitch, i);
    v2<T>* us = i == 0 ? A.u0 : gt_pick1(A.u, i);
    const int pu = i == 0 ? L.pitch : gt_pick1(A.pitch, i);
    gt_level_setup(L, X, tb);
    if (i > 0 || A.zero) {
#pragma unroll
      for (int q = 0; q < NP; ++q) {
        int k, j;
        if (gt_node(q, m, k, j)) us[(size_t)k * pu + j] = mk<T>(0, 0);
      }
    }
    for (int it = 0; it < A.nu1; ++it) gt_gmres3<T, NP>(L, X, tb, red, H, ys, us, pu, f, pf);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NP; ++q) {
      int k, j;
      if (gt_node(q, m, k, j)) X[k * GT_W + j] = us[(size_t)k * pu + j];
    }
    __syncthreads();
    v2<T> r[NP];
#pragma unroll
    for (int q = 0; q < NP; ++q) {
      int k, j;
      r[q] = mk<T>(0, 0);
      if (gt_node(q, m, k, j)) r[q] = csub(f[(size_t)k * pf + j], gt_apply(L, X, tb, k, j));
    }
    gt_store<T, NP>(X, r, m);
    const int nc = n / 2, mc = nc - 1;
    v2<T>* fc = gt_pick1(A.f, i + 1);
    const int pcn = gt_pick1(A.pitch, i + 1);
    for (int idx = tid; idx < mc * mc; idx += GT_THREADS) {
      const int K = idx / mc + 1, J = idx % mc + 1;
      v2<T> acc = mk<T>(0, 0);
#pragma unroll
      for (int a = -1; a <= 1; ++a)
#pragma unroll
        for (int b = -1; b <= 1; ++b) {
          const v2<T> rv = X[(2 * K + a) * GT_W + 2 * J + b];
          const T wgt = T((a == 0 ? 2 : 1) * (b == 0 ? 2 : 1));
          acc = mk<T>(acc.x + wgt * rv.x, acc.y + wgt * rv.y);
        }
      fc[(size_t)K * pcn + J] = cscale(acc, T(1.0 / 16.0));
    }
  }
  // coarsest level: u_c = Ainv f_c, one wave per row (k_coarse_solve), into X
  {
    const int nc = A.nc, mc = nc - 1, N = mc * mc;
    const v2<T>* fc = gt_pick1(A.f, A.nl);
    const int pc = gt_pick1(A.pitch, A.nl);
    __syncthreads();                             // every restriction write of f_c is visible
    const int w = tid >> 6, lane = tid & 63;
    for (int i = tid; i < (nc + 1) * (nc + 1); i += GT_THREADS) {
      const int k = i / (nc + 1), j = i % (nc + 1);
      if (k == 0 || k == nc || j == 0 || j == nc) X[k * GT_W + j] = mk<T>(0, 0);
    }
    for (int row = w; row < N; row += GT_WAVES) {
      double sr = 0, si = 0;
      const double2* Ar = A.Ainv + (size_t)row * N;
      for (int c = lane; c < N; c += 64) {
        const int k = c / mc + 1, j = c % mc + 1;
        v2<double> fv = cvt<double>(fc[(size_t)k * pc + j]);
        double2 a = Ar[c];
        sr += a.x * fv.x - a.y * fv.y;
        si += a.x * fv.y + a.y * fv.x;
      }
      sr = wave_sum(sr);
      si = wave_sum(si);
      if (lane == 0) X[(row / mc + 1) * GT_W + row % mc + 1] = mk<T>((T)sr, (T)si);
    }
  }
  // up: bilinear prolongation of the coarse correction, post-smoothing
  for (int i = A.nl - 1; i >= 0; --i) {
    const Level<T> L = gt_pick(A.L, i);
    const int n = L.n, m = n - 1;
    const v2<T>* f = i == 0 ? A.f0 : gt_pick1(A.f, i);
    const int pf = i == 0 ? L.pitch : gt_pick1(A.pitch, i);
    v2<T>* us = i == 0 ? A.u0 : gt_pick1(A.u, i);
    const int pu = i == 0 ? L.pitch : gt_pick1(A.pitch, i);
    __syncthreads();                             // the coarse correction in X is complete
#pragma unroll
    for (int q = 0; q < NP; ++q) {
      int k, j;
      if (gt_node(q, m, k, j)) {
        const int J0 = j >> 1, J1 = (j + 1) >> 1, K0 = k >> 1, K1 = (k + 1) >> 1;
        const v2<T> s = cadd(cadd(X[K0 * GT_W + J0], X[K0 * GT_W + J1]), cadd(X[K1 * GT_W + J0], X[K1 * GT_W + J1]));
        const size_t idx = (size_t)k * pu + j;
        us[idx] = cadd(us[idx], cscale(s, T(0.25)));
      }
    }
    gt_level_setup(L, X, tb);
    for (int it = 0; it < A.nu2; ++it) gt_gmres3<T, NP>(L, X, tb, red, H, ys, us, pu, f, pf);
    if (i > 0) {
      // the next finer level's coarse correction: this level's iterate in X
      __syncthreads();
#pragma unroll
      for (int q = 0; q < NP; ++q) {
        int k, j;
        if (gt_node(q, m, k, j)) X[k * GT_W + j] = us[(size_t)k * pu + j];
      }
    }
  }
}

template <typename T>
void launch_gs_tail(hipStream_t s, const GsTailArgs<T>& A) {
  // nodes per thread: enough for the top level (n = 64: 3969 nodes, 8 per
  // thread; n <= 32: 961, 2 per thread)
  const int m = A.L[0].n - 1;
  if (m * m <= 2 * GT_THREADS)
    hipLaunchKernelGGL((k_gs_tail<T, 2>), dim3(1), dim3(GT_THREADS), 0, s, A);
  else
    hipLaunchKernelGGL((k_gs_tail<T, (GT_MAX_N * GT_MAX_N + GT_THREADS - 1) / GT_THREADS>), dim3(1),
                       dim3(GT_THREADS), 0, s, A);
}
template void launch_gs_tail<double>(hipStream_t, const GsTailArgs<double>&);
template void launch_gs_tail<float>(hipStream_t, const GsTailArgs<float>&);

// ----------------------------------------------------------------------------
// BiCGSTAB outer loop (MGC_BICGSTAB), one iteration:
//   p = r + beta (p - omega v)                              k_bicg_p
//   p^ = B p  (one MG-CCCS cycle);  v = A p^, r~^H v        k_apply_dot (J = 1)
//   alpha = rho / r~^H v;  s = r - alpha v, ||s||^2         k_bicg_s
//   s^ = B s;  t = A s^, s^H t, ||t||^2                     k_apply_dot (J = 1)
//   omega = conj(s^H t) / ||t||^2;  u += alpha p^ + omega s^;  r = s - omega t;
//   r~^H r, ||r||^2 (if ||s|| already meets the tolerance: u += alpha p^, r = s)
//                                                           k_bicg_x
//   rho' = r~^H r;  beta = (rho'/rho)(alpha/omega);  rho = rho'   k_bicg_rho
// Scalars live on the device (BS_* slots below); every block that needs a
// scalar sums the producer's per-block partials itself in the same fixed
// order, so all blocks agree bit for bit.  The vectors are zero outside the
// interior, so the flat passes sweep the padded array.
enum { BS_RHO = 0, BS_ALPHA = 2, BS_OMEGA = 4, BS_BETA = 6, BS_RR = 8, BS_SS = 9, BS_CONV = 10 };
__global__ void k_bicg_init(double* bs, const double* nrm2) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  bs[BS_RHO] = nrm2[0];                        // r~ = r: rho = ||r||^2
  bs[BS_RHO + 1] = 0.0;
  bs[BS_ALPHA] = bs[BS_OMEGA] = 1.0;
  bs[BS_ALPHA + 1] = bs[BS_OMEGA + 1] = 0.0;
  bs[BS_BETA] = bs[BS_BETA + 1] = 0.0;         // p = v = 0 at the start
  bs[BS_RR] = nrm2[0];
  bs[BS_SS] = 0.0;
  bs[BS_CONV] = 0.0;
}
// p32, s32 (nullable): the new vector also rounded to FP32 (the FP32 cycle's
// input, same pitch)
__global__ void __launch_bounds__(AB) k_bicg_p(size_t Nf, const double2* __restrict__ r,
                                               const double2* __restrict__ v, double2* __restrict__ p,
                                               float2* __restrict__ p32, const double* __restrict__ bs) {
  const double2 beta = make_double2(bs[BS_BETA], bs[BS_BETA + 1]);
  const double2 om = make_double2(bs[BS_OMEGA], bs[BS_OMEGA + 1]);
  for (size_t i = (size_t)blockIdx.x * AB + threadIdx.x; i < Nf; i += (size_t)gridDim.x * AB) {
    const double2 pv = p[i], vv = v[i], rv = r[i];
    const double2 d = make_double2(pv.x - (om.x * vv.x - om.y * vv.y), pv.y - (om.x * vv.y + om.y * vv.x));
    const double2 pn = make_double2(rv.x + (beta.x * d.x - beta.y * d.y), rv.y + (beta.x * d.y + beta.y * d.x));
    p[i] = pn;
    if (p32) p32[i] = make_float2((float)pn.x, (float)pn.y);
  }
}
__global__ void __launch_bounds__(AB) k_bicg_s(size_t Nf, const double* __restrict__ pin, int nbin,
                                               double* __restrict__ bs, const double2* __restrict__ r,
                                               const double2* __restrict__ v, double2* __restrict__ sv,
                                               float2* __restrict__ s32, double* __restrict__ pout) {
  __shared__ double dsum[3];
  finish_sum_nt<AB>(pin, nbin, 3, dsum);       // r~^H v, ||v||^2
  const double2 rho = make_double2(bs[BS_RHO], bs[BS_RHO + 1]);
  const double2 alpha = cdiv(rho, make_double2(dsum[0], dsum[1]));
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    bs[BS_ALPHA] = alpha.x;
    bs[BS_ALPHA + 1] = alpha.y;
  }
  double acc[1] = {0.0};
  for (size_t i = (size_t)blockIdx.x * AB + threadIdx.x; i < Nf; i += (size_t)gridDim.x * AB) {
    const double2 rv = r[i], vv = v[i];
    const double2 sx = make_double2(rv.x - (alpha.x * vv.x - alpha.y * vv.y), rv.y - (alpha.x * vv.y + alpha.y * vv.x));
    sv[i] = sx;
    if (s32) s32[i] = make_float2((float)sx.x, (float)sx.y);
    acc[0] += sx.x * sx.x + sx.y * sx.y;
  }
  double tot[1];
  block_sum<1>(acc, tot);
  if (threadIdx.x == 0) pout[blockIdx.x] = tot[0];
}
template <typename TZ>
__global__ void __launch_bounds__(256) k_bicg_x(int n, int pitch, const double* __restrict__ pin, int nbin,
                                                const double* __restrict__ ps, int nbs, double tol2,
                                                double* __restrict__ bs, const v2<TZ>* __restrict__ ph,
                                                const v2<TZ>* __restrict__ sh, const double2* __restrict__ sv,
                                                const double2* __restrict__ t, const double2* __restrict__ rt,
                                                double2* __restrict__ r, double2* __restrict__ x,
                                                double* __restrict__ pout) {
  __shared__ double dsum[3], ssum[1];
  finish_sum_nt<256>(pin, nbin, 3, dsum);      // s^H t, ||t||^2
  finish_sum_nt<256>(ps, nbs, 1, ssum);        // ||s||^2
  const bool conv = ssum[0] <= tol2;
  const double2 alpha = make_double2(bs[BS_ALPHA], bs[BS_ALPHA + 1]);
  // t^H s = conj(s^H t)
  const double2 omega = conv ? make_double2(0.0, 0.0) : make_double2(dsum[0] / dsum[2], -dsum[1] / dsum[2]);
  if (flat_block() == 0 && threadIdx.x == 0) {
    bs[BS_OMEGA] = omega.x;
    bs[BS_OMEGA + 1] = omega.y;
    bs[BS_SS] = ssum[0];
    bs[BS_CONV] = conv ? 1.0 : 0.0;
  }
  double acc[3] = {0.0, 0.0, 0.0};
  MGC_NODE_LOOP(n, k, j) {
    const size_t idx = (size_t)k * pitch + j;
    const v2<double> a = cvt<double>(ph[idx]);
    double2 xv = x[idx];
    const double2 sx = sv[idx];
    double2 rn;
    if (conv) {
      xv = make_double2(xv.x + (alpha.x * a.x - alpha.y * a.y), xv.y + (alpha.x * a.y + alpha.y * a.x));
      rn = sx;
    } else {
      const v2<double> b = cvt<double>(sh[idx]);
      const double2 tv = t[idx];
      xv = make_double2(xv.x + (alpha.x * a.x - alpha.y * a.y) + (omega.x * b.x - omega.y * b.y),
                        xv.y + (alpha.x * a.y + alpha.y * a.x) + (omega.x * b.y + omega.y * b.x));
      rn = make_double2(sx.x - (omega.x * tv.x - omega.y * tv.y), sx.y - (omega.x * tv.y + omega.y * tv.x));
    }
    x[idx] = xv;
    r[idx] = rn;
    const double2 w = rt[idx];
    acc[0] += w.x * rn.x + w.y * rn.y;         // r~^H r
    acc[1] += w.x * rn.y - w.y * rn.x;
    acc[2] += rn.x * rn.x + rn.y * rn.y;
  }
  double tot[3];
  block_sum<3>(acc, tot);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < 3; ++q) pout[(size_t)flat_block() * 3 + q] = tot[q];
  }
}
__global__ void __launch_bounds__(256) k_bicg_rho(const double* __restrict__ pin, int nbin, double* __restrict__ bs,
                                                  double* __restrict__ rep) {
  __shared__ double dsum[3];
  finish_sum_nt<256>(pin, nbin, 3, dsum);
  if (threadIdx.x == 0) {
    const double2 rn = make_double2(dsum[0], dsum[1]);
    const double2 rho = make_double2(bs[BS_RHO], bs[BS_RHO + 1]);
    const double2 alpha = make_double2(bs[BS_ALPHA], bs[BS_ALPHA + 1]);
    const double2 omega = make_double2(bs[BS_OMEGA], bs[BS_OMEGA + 1]);
    const double2 beta = bs[BS_CONV] != 0.0 ? make_double2(0.0, 0.0) : cmul(cdiv(rn, rho), cdiv(alpha, omega));
    bs[BS_BETA] = beta.x;
    bs[BS_BETA + 1] = beta.y;
    bs[BS_RHO] = rn.x;
    bs[BS_RHO + 1] = rn.y;
    bs[BS_RR] = dsum[2];
    rep[0] = dsum[2];
    rep[1] = bs[BS_SS];
    rep[2] = bs[BS_CONV];
  }
}

// x2 side of the single-ionisation sweep: F2[k][2q + part] = t_k * (Re, Im)
// of the bound state q at node k (t the trapezoid weights of the real region:
// h, h/2 at j0), zero outside 1 .. top and for the padding pairs.
__global__ void __launch_bounds__(256) k_bound_weights(int n, int top, int j0, double h, int nstates, int pp,
                                                      const double2* __restrict__ tab, double* __restrict__ F2) {
  const size_t total = (size_t)(n + 1) * pp;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (size_t)gridDim.x * 256) {
    const int k = (int)(i / pp), c = (int)(i - (size_t)k * pp), q = c >> 1;
    double v = 0.0;
    if (k >= 1 && k <= top && q < nstates) {
      const double2 b = tab[(size_t)q * (n + 1) + k];
      v = (k == j0 ? 0.5 * h : h) * ((c & 1) ? b.y : b.x);
    }
    F2[i] = v;
  }
}
void launch_bound_weights(hipStream_t s, int n, int top, int j0, double h, int nstates, int pp, const double2* tab,
                          double* F2) {
  const size_t total = (size_t)(n + 1) * pp;
  const int blocks = (int)std::min<size_t>(1024, (total + 255) / 256);
  hipLaunchKernelGGL(k_bound_weights, dim3(blocks), dim3(256), 0, s, n, top, j0, h, nstates, pp, tab, F2);
}

template <typename T>
__global__ void __launch_bounds__(256) k_add(int n, int pitch, const v2<T>* __restrict__ e, v2<T>* __restrict__ u) {
  MGC_NODE_LOOP(n, k, j) {
    const size_t idx = (size_t)k * pitch + j;
    u[idx] = cadd(u[idx], e[idx]);
  }
}
template <typename T>
void launch_add(hipStream_t s, int n, int pitch, const void* e, void* u) {
  hipLaunchKernelGGL((k_add<T>), vec_grid(n), dim3(256), 0, s, n, pitch, (const v2<T>*)e, (v2<T>*)u);
}
template void launch_add<double>(hipStream_t, int, int, const void*, void*);
template void launch_add<float>(hipStream_t, int, int, const void*, void*);

template <typename T>
void launch_gmres3_smooth(hipStream_t s, const Level<T>& L, void* u, const void* f, void* V, size_t stride, double* st,
                          double* part) {
  const int n = L.n, p = L.pitch;
  const dim3 vg = vec_grid(n);
  const int nbv = vec_blocks(n), nbs = stencil_blocks(n);
  double* pa = part;                       // dots of the Arnoldi step: nbv x 6
  double* pb = part + (size_t)nbv * 2 * GS_M;   // squared norms: max(nbv, 2 nbs)
  v2<T>* Vt = (v2<T>*)V;
  hipLaunchKernelGGL((k_stencil<T, T, T, T>), stencil_grid(n), dim3(SX, SY), 0, s, L, (const v2<T>*)u,
                     (const v2<T>*)f, Vt, 0, pb);
  hipLaunchKernelGGL((k_gs_normalize<T>), vg, dim3(256), 0, s, n, p, Vt, (const double*)pb, nbs, 2, st, GS_BETA);
#define MGC_GS_STEP(JJ)                                                                                       \
  hipLaunchKernelGGL((k_gs_arnoldi<T, JJ>), vg, dim3(256), 0, s, L, Vt, stride, pa);                          \
  hipLaunchKernelGGL((k_gs_orth<T, JJ>), vg, dim3(256), 0, s, n, p, Vt, stride, (const double*)pa, nbv, st, pb); \
  hipLaunchKernelGGL((k_gs_normalize<T>), vg, dim3(256), 0, s, n, p, Vt + (size_t)JJ * stride, (const double*)pb, \
                     nbv, 1, st, 2 * ((JJ - 1) * (GS_M + 1) + JJ));
  MGC_GS_STEP(1)
  MGC_GS_STEP(2)
  MGC_GS_STEP(3)
#undef MGC_GS_STEP
  hipLaunchKernelGGL(k_gs_solve, dim3(1), dim3(1), 0, s, st);
  hipLaunchKernelGGL((k_gs_update<T>), vg, dim3(256), 0, s, n, p, (const v2<T>*)Vt, stride, (const double*)st,
                     (v2<T>*)u);
}
template void launch_gmres3_smooth<double>(hipStream_t, const Level<double>&, void*, const void*, void*, size_t,
                                           double*, double*);
template void launch_gmres3_smooth<float>(hipStream_t, const Level<float>&, void*, const void*, void*, size_t,
                                          double*, double*);
int gmres3_part_doubles(int n) { return vec_blocks(n) * 2 * GS_M + std::max(vec_blocks(n), 2 * stencil_blocks(n)); }

void launch_bicg_init(hipStream_t s, double* bs, const double* nrm2) {
  hipLaunchKernelGGL(k_bicg_init, dim3(1), dim3(1), 0, s, bs, nrm2);
}
void launch_bicg_p(hipStream_t s, int n, int pitch, const double2* r, const double2* v, double2* p,
                   float2* p32, const double* bs) {
  hipLaunchKernelGGL(k_bicg_p, dim3(axpy_blocks(n, pitch)), dim3(AB), 0, s, (size_t)(n + 1) * pitch, r, v, p, p32,
                     bs);
}
void launch_bicg_s(hipStream_t s, int n, int pitch, const double* part_ad, double* bs, const double2* r,
                   const double2* v, double2* sv, float2* s32, double* part_s) {
  const ApplyGrid ag = apply_dot_grid(n);
  hipLaunchKernelGGL(k_bicg_s, dim3(axpy_blocks(n, pitch)), dim3(AB), 0, s, (size_t)(n + 1) * pitch, part_ad,
                     (int)(ag.grid.x * ag.grid.y), bs, r, v, sv, s32, part_s);
}
template <typename TZ>
void launch_bicg_x(hipStream_t s, int n, int pitch, const double* part_ad, const double* part_s, double tol2,
                   double* bs, const void* ph, const void* sh, const double2* sv, const double2* t, const double2* rt,
                   double2* r, double2* x, double* part_x) {
  const ApplyGrid ag = apply_dot_grid(n);
  hipLaunchKernelGGL((k_bicg_x<TZ>), vec_grid(n), dim3(256), 0, s, n, pitch, part_ad, (int)(ag.grid.x * ag.grid.y),
                     part_s, axpy_blocks(n, pitch), tol2, bs, (const v2<TZ>*)ph, (const v2<TZ>*)sh, sv, t, rt, r, x,
                     part_x);
}
template void launch_bicg_x<double>(hipStream_t, int, int, const double*, const double*, double, double*, const void*,
                                    const void*, const double2*, const double2*, const double2*, double2*, double2*,
                                    double*);
template void launch_bicg_x<float>(hipStream_t, int, int, const double*, const double*, double, double*, const void*,
                                   const void*, const double2*, const double2*, const double2*, double2*, double2*,
                                   double*);
void launch_bicg_rho(hipStream_t s, int n, const double* part_x, double* bs, double* rep) {
  hipLaunchKernelGGL(k_bicg_rho, dim3(1), dim3(256), 0, s, part_x, vec_blocks(n), bs, rep);
}

void launch_zeta_sweep(hipStream_t s, int n, int pitch, int top, int pp, const double2* tm, const double* F1T,
                       const double* F2T, const double2* u, const double2* chi, double* part, double* out) {
  hipLaunchKernelGGL(k_zeta_sweep_part, dim3((top + SWR - 1) / SWR, SWJ), dim3(pp), 0, s, n, pitch, top, pp, tm,
                     F1T, F2T, u, chi, part);
  hipLaunchKernelGGL(k_zeta_sweep_sum, dim3((2 * pp + SWQ - 1) / SWQ), dim3(256), 0, s, zeta_sweep_blocks(top),
                     2 * pp, (const double*)part, out);
}

}  // namespace mgc
