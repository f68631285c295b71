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
#include "device.h"
#include "launch.h"

namespace mgc {

// ----------------------------------------------------------------------------
// complex helpers
template <typename T> __device__ __forceinline__ v2<T> mk(T x, T y) { v2<T> r; r.x = x; r.y = y; return r; }
#define MGC_CPLX_OPS(V, T)                                                                  \
  __device__ __forceinline__ V cadd(V a, V b) { return mk<T>(a.x + b.x, a.y + b.y); }        \
  __device__ __forceinline__ V csub(V a, V b) { return mk<T>(a.x - b.x, a.y - b.y); }        \
  __device__ __forceinline__ V cmul(V a, V b) {                                             \
    return mk<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);                             \
  }                                                                                         \
  /* acc + a*b */                                                                           \
  __device__ __forceinline__ V cfma(V acc, V a, V b) {                                      \
    return mk<T>(acc.x + a.x * b.x - a.y * b.y, acc.y + a.x * b.y + a.y * b.x);             \
  }                                                                                         \
  __device__ __forceinline__ V cscale(V a, T s) { return mk<T>(a.x * s, a.y * s); }          \
  __device__ __forceinline__ V cdiv(V a, V b) {                                             \
    T inv = T(1) / (b.x * b.x + b.y * b.y);                                                 \
    return mk<T>((a.x * b.x + a.y * b.y) * inv, (a.y * b.x - a.x * b.y) * inv);             \
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

template <typename T> __device__ __forceinline__ T shfl_xor_t(T v, int m) { return __shfl_xor(v, m, 64); }

__device__ __forceinline__ double wave_sum(double v) {
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// Operator diagonal at (k, j): px_j + py_k + tm_max(j,k) - E
template <typename T>
__device__ __forceinline__ v2<T> diag_at(const Level<T>& L, int k, int j) {
  v2<T> d = cadd(cadd(L.px[j], L.py[k]), L.tm[j > k ? j : k]);
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
    for (int r = 0; r < ROWS; ++r) {
      const int k = k0 + r;
      if (k >= n) break;
      v2<T> Au = apply_at<T>(L, u, k, j);
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
constexpr int S1CX = 32, S1CY = 8;                       // coarse points per block
constexpr int S1W = 2 * S1CX + 3, S1H = 2 * S1CY + 3;    // u' tile (fine nodes)
constexpr int S1RW = 2 * S1CX + 1, S1RH = 2 * S1CY + 1;  // residual tile

template <typename T>
__global__ void __launch_bounds__(256) k_s1_zero(Level<T> L, const v2<T>* __restrict__ f,
                                                 const double* __restrict__ fs, T omega,
                                                 v2<T>* __restrict__ fc, int pitch_c) {
  __shared__ v2<T> up[S1H][S1W];
  __shared__ v2<T> fl[S1H][S1W];
  __shared__ v2<T> rl[S1RH][S1RW];
  const int n = L.n, p = L.pitch, nc = n / 2;
  const int tid = threadIdx.x + 64 * threadIdx.y;
  const int J0 = 1 + blockIdx.x * S1CX, K0 = 1 + blockIdx.y * S1CY;
  const int c0 = 2 * J0 - 2, r0 = 2 * K0 - 2;             // fine origin of the u' tile
  const T sc = fs ? (T)*fs : T(1);
  for (int idx = tid; idx < S1H * S1W; idx += 256) {
    const int rr = idx / S1W, cc = idx % S1W;
    const int k = r0 + rr, j = c0 + cc;
    v2<T> fv = mk<T>(0, 0), uv = mk<T>(0, 0);
    if (j > 0 && j < n && k > 0 && k < n) {
      fv = cscale(f[(size_t)k * p + j], sc);
      uv = cscale(cdiv(fv, diag_at(L, k, j)), omega);
    }
    up[rr][cc] = uv;
    fl[rr][cc] = fv;
  }
  __syncthreads();
  for (int idx = tid; idx < S1RH * S1RW; idx += 256) {
    const int rr = 1 + idx / S1RW, cc = 1 + idx % S1RW;
    const int k = r0 + rr, j = c0 + cc;
    v2<T> r = mk<T>(0, 0);
    if (j > 0 && j < n && k > 0 && k < n) {
      v2<T> acc = cmul(diag_at(L, k, j), up[rr][cc]);
      acc = cfma(acc, L.a[j], up[rr][cc - 1]);
      acc = cfma(acc, L.c[j], up[rr][cc + 1]);
      acc = cfma(acc, L.a[k], up[rr - 1][cc]);
      acc = cfma(acc, L.c[k], up[rr + 1][cc]);
      r = csub(fl[rr][cc], acc);
    }
    rl[rr - 1][cc - 1] = r;
  }
  __syncthreads();
  const int J = J0 + threadIdx.x % S1CX, K = K0 + (tid / S1CX);
  if (tid < S1CX * S1CY && J < nc && K < nc) {
    const int cr = 2 * (K - K0) + 1, ccn = 2 * (J - J0) + 1;   // centre in rl
    v2<T> acc = mk<T>(0, 0);
#pragma unroll
    for (int a = -1; a <= 1; ++a)
#pragma unroll
      for (int b = -1; b <= 1; ++b) {
        const T w = T((a == 0 ? 2 : 1) * (b == 0 ? 2 : 1));
        v2<T> r = rl[cr + a][ccn + b];
        acc = mk<T>(acc.x + w * r.x, acc.y + w * r.y);
      }
    fc[(size_t)K * pitch_c + J] = cscale(acc, T(1.0 / 16.0));
  }
}

constexpr int S2TX = 64, S2TY = 16;
constexpr int S2W = S2TX + 2, S2H = S2TY + 2;

template <typename T>
__global__ void __launch_bounds__(256) k_s2_zero(Level<T> L, const v2<T>* __restrict__ f,
                                                 const double* __restrict__ fs, T omega,
                                                 const v2<T>* __restrict__ ec, int pitch_c,
                                                 v2<T>* __restrict__ u) {
  __shared__ v2<T> wl[S2H][S2W];
  __shared__ v2<T> fl[S2H][S2W];
  const int n = L.n, p = L.pitch, nc = n / 2;
  const int tid = threadIdx.x + 64 * threadIdx.y;
  const int j0 = 1 + blockIdx.x * S2TX - 1, k0 = 1 + blockIdx.y * S2TY - 1;   // tile origin (halo)
  const T sc = fs ? (T)*fs : T(1);
  for (int idx = tid; idx < S2H * S2W; idx += 256) {
    const int rr = idx / S2W, cc = idx % S2W;
    const int k = k0 + rr, j = j0 + cc;
    v2<T> fv = mk<T>(0, 0), wv = mk<T>(0, 0);
    if (j > 0 && j < n && k > 0 && k < n) {
      fv = cscale(f[(size_t)k * p + j], sc);
      wv = cscale(cdiv(fv, diag_at(L, k, j)), omega);
      const int Ja = j >> 1, Jb = (j + 1) >> 1, Ka = k >> 1, Kb = (k + 1) >> 1;
      v2<T> s = cadd(cadd(ldf<T>(ec, pitch_c, Ka, Ja, nc), ldf<T>(ec, pitch_c, Ka, Jb, nc)),
                     cadd(ldf<T>(ec, pitch_c, Kb, Ja, nc), ldf<T>(ec, pitch_c, Kb, Jb, nc)));
      wv = cadd(wv, cscale(s, T(0.25)));
    }
    wl[rr][cc] = wv;
    fl[rr][cc] = fv;
  }
  __syncthreads();
  const int cc = 1 + threadIdx.x;
  const int j = j0 + cc;
  if (j >= n) return;
  for (int q = 0; q < S2TY / 4; ++q) {
    const int rr = 1 + threadIdx.y + 4 * q;
    const int k = k0 + rr;
    if (k >= n) break;
    v2<T> d = diag_at(L, k, j);
    v2<T> acc = cmul(d, wl[rr][cc]);
    acc = cfma(acc, L.a[j], wl[rr][cc - 1]);
    acc = cfma(acc, L.c[j], wl[rr][cc + 1]);
    acc = cfma(acc, L.a[k], wl[rr - 1][cc]);
    acc = cfma(acc, L.c[k], wl[rr + 1][cc]);
    v2<T> res = csub(fl[rr][cc], acc);
    u[(size_t)k * p + j] = cadd(wl[rr][cc], cscale(cdiv(res, d), omega));
  }
}

// ----------------------------------------------------------------------------
// CCCS.  Step 1: residual r = f - A u written to rbuf, together with
// rho^A[k][i] = sum_j w_j phi_i(j) r[k][j] -- one wave per row k.
template <typename T, int MC>
__global__ void __launch_bounds__(64) k_cccs_resid_rhoA(Level<T> L, const v2<T>* __restrict__ u,
                                                        const v2<T>* __restrict__ f,
                                                        const double* __restrict__ fs,
                                                        v2<T>* __restrict__ rbuf, ChanTab<T> ch,
                                                        v2<T>* __restrict__ rhoA) {
  const int k = 1 + blockIdx.x;
  const int n = L.n, p = L.pitch, M = ch.M;
  const T sc = fs ? (T)*fs : T(1);
  v2<T> acc[MC];
#pragma unroll
  for (int i = 0; i < MC; ++i) acc[i] = mk<T>(0, 0);
  for (int j = 1 + threadIdx.x; j < n; j += 64) {
    v2<T> r = csub(cscale(f[(size_t)k * p + j], sc), apply_at<T>(L, u, k, j));
    rbuf[(size_t)k * p + j] = r;
#pragma unroll
    for (int i = 0; i < MC; ++i)
      if (i < M) acc[i] = cfma(acc[i], ch.wphi[(size_t)i * (n + 1) + j], r);
  }
#pragma unroll
  for (int i = 0; i < MC; ++i) {
    if (i < M) {
      T x = acc[i].x, y = acc[i].y;
      for (int m = 32; m >= 1; m >>= 1) { x += shfl_xor_t(x, m); y += shfl_xor_t(y, m); }
      if (threadIdx.x == 0) rhoA[(size_t)k * M + i] = mk<T>(x, y);
    }
  }
}

// Step 2: column projections rho^B[j][l] = sum_k w_k varphi_l(k) r[k][j],
// partial over row chunks of CHR rows: partB[chunk][j][l].
constexpr int CHR = 64;
template <typename T, int LC>
__global__ void __launch_bounds__(64) k_cccs_rhoB_part(int n, int pitch, const v2<T>* __restrict__ rbuf,
                                                       ChanTab<T> ch, v2<T>* __restrict__ partB) {
  const int j = 1 + blockIdx.x * 64 + threadIdx.x;
  const int kb = 1 + blockIdx.y * CHR;
  const int Lc = ch.L;
  if (j >= n) return;
  v2<T> acc[LC];
#pragma unroll
  for (int l = 0; l < LC; ++l) acc[l] = mk<T>(0, 0);
  const int ke = min(kb + CHR, n);
  for (int k = kb; k < ke; ++k) {
    v2<T> r = rbuf[(size_t)k * pitch + j];
#pragma unroll
    for (int l = 0; l < LC; ++l)
      if (l < Lc) acc[l] = cfma(acc[l], ch.wvphi[(size_t)l * (n + 1) + k], r);
  }
  v2<T>* out = partB + ((size_t)blockIdx.y * (n + 1) + j) * Lc;
#pragma unroll
  for (int l = 0; l < LC; ++l)
    if (l < Lc) out[l] = acc[l];
}

// Step 3: rho^B from the partials (fixed order).
template <typename T>
__global__ void k_cccs_rhoB_sum(int n, int nchunks, int Lc, const v2<T>* __restrict__ partB,
                                v2<T>* __restrict__ rhoB) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;   // (j-1)*Lc + l
  if (idx >= (n - 1) * Lc) return;
  const int j = 1 + idx / Lc, l = idx % Lc;
  v2<T> s = mk<T>(0, 0);
  for (int c = 0; c < nchunks; ++c) s = cadd(s, partB[((size_t)c * (n + 1) + j) * Lc + l]);
  rhoB[(size_t)j * Lc + l] = s;
}

// Step 4: coupling coefficients c[i][l] = sum_k w_k varphi_l(k) rho^A[k][i]
// (eq. coefficients).  One block; thread per (i, l) pair, then LDS partial
// reduction over k-slices.
template <typename T>
__global__ void __launch_bounds__(256) k_cccs_coef(int n, ChanTab<T> ch, const v2<T>* __restrict__ rhoA,
                                                   v2<T>* __restrict__ coef) {
  const int M = ch.M, Lc = ch.L, P = M * Lc;
  const int nslice = 256 / P;                    // >= 1 because P <= 256
  const int t = threadIdx.x;
  const int pair = t % P, slice = t / P;
  __shared__ double sre[256], sim[256];
  double xr = 0, xi = 0;
  if (slice < nslice) {
    const int i = pair / Lc, l = pair % Lc;
    for (int k = 1 + slice; k < n; k += nslice) {
      v2<T> a = ch.wvphi[(size_t)l * (n + 1) + k], b = rhoA[(size_t)k * M + i];
      xr += (double)a.x * b.x - (double)a.y * b.y;
      xi += (double)a.x * b.y + (double)a.y * b.x;
    }
  }
  sre[t] = xr;
  sim[t] = xi;
  __syncthreads();
  if (t < P) {
    double sr = 0, si = 0;
    for (int s = 0; s < nslice; ++s) { sr += sre[s * P + t]; si += sim[s * P + t]; }
    coef[t] = mk<T>((T)sr, (T)si);
  }
}

// Wave-level dense mat-vec y = A x for an R x R row-major matrix (R <= 32),
// x and y in LDS.  g = 64 / next_pow2(R) lanes share a row.
template <typename T>
__device__ __forceinline__ void wave_matvec(int R, int gsh, const v2<T>* __restrict__ A,
                                            const v2<T>* x, v2<T>* y) {
  const int lane = threadIdx.x & 63;
  const int g = 1 << gsh;
  const int i = lane >> gsh, part = lane & (g - 1);
  T sr = 0, si = 0;
  if (i < R) {
    for (int m = part; m < R; m += g) {
      v2<T> a = A[i * R + m], b = x[m];
      sr += a.x * b.x - a.y * b.y;
      si += a.x * b.y + a.y * b.x;
    }
  }
  for (int s = 1; s < g; s <<= 1) { sr += shfl_xor_t(sr, s); si += shfl_xor_t(si, s); }
  __syncthreads();   // every lane finished reading x (x may alias y's buffer)
  if (i < R && part == 0) y[i] = mk<T>(sr, si);
  __syncthreads();
}

__device__ __forceinline__ int pow2_shift_for(int R) {
  int r2 = 1;
  while (r2 < R) r2 <<= 1;
  int g = 64 / r2;
  int s = 0;
  while ((1 << s) < g) ++s;
  return s;
}

// Step 5: chunk-local block LU solves of both channel systems.  Block = one
// wave; blockIdx.x = chunk, blockIdx.y = system (0: A, functions of x2 with
// x1 channels; 1: B, functions of x1 with x2 channels).  The right-hand sides
// follow the uniqueness convention (Remark 4):
//   r^A_i(k) = rho^A_i(k) - sum_{l > i} c_il varphi_l(k)
//   r^B_l(j) = rho^B_l(j) - sum_{m >= l} c_ml phi_m(j)
template <typename T>
__global__ void __launch_bounds__(64) k_cccs_local(ChanSys<T> SA, ChanSys<T> SB, ChanTab<T> ch,
                                                   int n, const v2<T>* __restrict__ rhoA,
                                                   const v2<T>* __restrict__ rhoB,
                                                   const v2<T>* __restrict__ coef,
                                                   v2<T>* __restrict__ gA, v2<T>* __restrict__ gB) {
  const bool isA = blockIdx.y == 0;
  const ChanSys<T>& S = isA ? SA : SB;
  const int p = blockIdx.x;
  if (p >= S.P) return;
  const int M = S.M, MM = M * M, Mo = isA ? ch.L : ch.M;  // Mo: channel count of the other axis
  const int s = S.start[p], e = S.start[p + 1] - 1;
  const int lane = threadIdx.x;
  const int gsh = pow2_shift_for(M);
  __shared__ v2<T> xv[32], yv[32];
  v2<T>* g = isA ? gA : gB;
  const v2<T>* rho = isA ? rhoA : rhoB;
  // forward sweep: Z_t = G_t (rhs_t - lo_t Z_{t-1})
  for (int t = s; t <= e; ++t) {
    const int node = t + 1;
    if (lane < M) {
      v2<T> v = rho[(size_t)node * M + lane];
      if (isA) {
        for (int l = lane + 1; l < Mo; ++l)   // b_il = c_il for l > i
          v = csub(v, cmul(coef[lane * Mo + l], ch.vphi[(size_t)l * (n + 1) + node]));
      } else {
        for (int m = lane; m < Mo; ++m)       // a_lm = c_ml for l <= m
          v = csub(v, cmul(coef[m * M + lane], ch.phi[(size_t)m * (n + 1) + node]));
      }
      if (t > s) v = csub(v, cmul(S.lo[t], yv[lane]));
      xv[lane] = v;
    }
    __syncthreads();
    wave_matvec<T>(M, gsh, S.G + (size_t)t * MM, xv, yv);
    if (lane < M) g[(size_t)t * M + lane] = yv[lane];
    __syncthreads();
  }
  // backward sweep: g_t = Z_t - up_t G_t g_{t+1}
  for (int t = e - 1; t >= s; --t) {
    if (lane < M) xv[lane] = yv[lane];
    __syncthreads();
    wave_matvec<T>(M, gsh, S.G + (size_t)t * MM, xv, yv);
    if (lane < M) {
      v2<T> z = g[(size_t)t * M + lane];
      v2<T> r = csub(z, cmul(S.up[t], yv[lane]));
      g[(size_t)t * M + lane] = r;
      yv[lane] = r;
    }
    __syncthreads();
  }
}

// Step 6: interface systems (one wave per system), unknowns Y_q = [B_q; T_{q+1}].
template <typename T>
__global__ void __launch_bounds__(64) k_cccs_iface(ChanSys<T> SA, ChanSys<T> SB,
                                                   const v2<T>* __restrict__ gA,
                                                   const v2<T>* __restrict__ gB,
                                                   v2<T>* __restrict__ YA, v2<T>* __restrict__ YB) {
  const bool isA = blockIdx.x == 0;
  const ChanSys<T>& S = isA ? SA : SB;
  const v2<T>* g = isA ? gA : gB;
  v2<T>* Y = isA ? YA : YB;
  const int M = S.M, R = 2 * M, RR = R * R, Q = S.P - 1;
  if (Q <= 0) return;
  const int lane = threadIdx.x;
  const int gsh = pow2_shift_for(R);
  __shared__ v2<T> xv[32], yv[32], zp[32];
  for (int q = 0; q < Q; ++q) {
    const int e_q = S.start[q + 1] - 1, s_n = S.start[q + 1];
    if (lane < M) {
      xv[lane] = g[(size_t)e_q * M + lane];
      xv[M + lane] = g[(size_t)s_n * M + lane];
    }
    __syncthreads();
    wave_matvec<T>(R, gsh, S.Rinv + (size_t)q * RR, xv, yv);     // Rinv_q rhs_q
    if (q > 0) {
      wave_matvec<T>(R, gsh, S.Rlo + (size_t)q * RR, zp, xv);    // Rlo_q Z_{q-1}
      if (lane < R) yv[lane] = csub(yv[lane], xv[lane]);
      __syncthreads();
    }
    if (lane < R) { Y[(size_t)q * R + lane] = yv[lane]; zp[lane] = yv[lane]; }
    __syncthreads();
  }
  for (int q = Q - 2; q >= 0; --q) {
    wave_matvec<T>(R, gsh, S.Rup + (size_t)q * RR, zp, xv);      // Rup_q Y_{q+1}
    if (lane < R) {
      v2<T> v = csub(Y[(size_t)q * R + lane], xv[lane]);
      Y[(size_t)q * R + lane] = v;
      zp[lane] = v;
    }
    __syncthreads();
  }
}

// Step 7: retrieval e_t = g_t - V_t T_{p+1} - W_t B_{p-1}; thread per (t, i).
template <typename T>
__global__ void __launch_bounds__(256) k_cccs_retrieve(ChanSys<T> SA, ChanSys<T> SB,
                                                       const v2<T>* __restrict__ gA,
                                                       const v2<T>* __restrict__ gB,
                                                       const v2<T>* __restrict__ YA,
                                                       const v2<T>* __restrict__ YB,
                                                       v2<T>* __restrict__ eA, v2<T>* __restrict__ eB) {
  const bool isA = blockIdx.y == 0;
  const ChanSys<T>& S = isA ? SA : SB;
  const int M = S.M, MM = M * M, R = 2 * M;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= S.N * M) return;
  const int t = idx / M, i = idx % M;
  const v2<T>* g = isA ? gA : gB;
  const v2<T>* Y = isA ? YA : YB;
  v2<T>* e = isA ? eA : eB;
  int p = 0;
  while (t >= S.start[p + 1]) ++p;
  v2<T> v = g[(size_t)t * M + i];
  if (p + 1 < S.P) {
    const v2<T>* Tn = Y + (size_t)p * R + M;
    for (int m = 0; m < M; ++m) v = csub(v, cmul(S.Vs[(size_t)t * MM + i * M + m], Tn[m]));
  }
  if (p > 0) {
    const v2<T>* Bp = Y + (size_t)(p - 1) * R;
    for (int m = 0; m < M; ++m) v = csub(v, cmul(S.Ws[(size_t)t * MM + i * M + m], Bp[m]));
  }
  e[(size_t)(t + 1) * M + i] = v;   // node index t+1
}

// Step 8: expansion u += sum_m eA[k][m] phi_m(j) + sum_l eB[j][l] varphi_l(k)
template <typename T, int MC>
__global__ void __launch_bounds__(256) k_cccs_expand(int n, int pitch, v2<T>* __restrict__ u,
                                                     ChanTab<T> ch, const v2<T>* __restrict__ eA,
                                                     const v2<T>* __restrict__ eB) {
  const int j = 1 + blockIdx.x * SX + threadIdx.x;
  const int k0 = 1 + (blockIdx.y * SY + threadIdx.y) * ROWS;
  if (j >= n) return;
  const int M = ch.M, Lc = ch.L;
  v2<T> ph[MC], eb[MC];
#pragma unroll
  for (int m = 0; m < MC; ++m) {
    ph[m] = (m < M) ? ch.phi[(size_t)m * (n + 1) + j] : mk<T>(0, 0);
    eb[m] = (m < Lc) ? eB[(size_t)j * Lc + m] : mk<T>(0, 0);
  }
  for (int r = 0; r < ROWS; ++r) {
    const int k = k0 + r;
    if (k >= n) break;
    const size_t idx = (size_t)k * pitch + j;
    v2<T> v = u[idx];
#pragma unroll
    for (int m = 0; m < MC; ++m) {
      if (m < M) v = cfma(v, eA[(size_t)k * M + m], ph[m]);
      if (m < Lc) v = cfma(v, eb[m], ch.vphi[(size_t)m * (n + 1) + k]);
    }
    u[idx] = v;
  }
}

// ----------------------------------------------------------------------------
// Vector kernels for the FP64 outer loop (grid-stride over interior nodes).
__device__ __forceinline__ void node_of(long t, int m, int& k, int& j) {
  k = (int)(t / m) + 1;
  j = (int)(t % m) + 1;
}

// part[b][q] = sum conj(W_q) Y over the block's nodes, q < J (J <= 32).
template <int JMAX>
__global__ void __launch_bounds__(256) k_multidot(int n, int pitch, size_t stride,
                                                  const double2* __restrict__ W, int J,
                                                  const double2* __restrict__ Y,
                                                  double* __restrict__ part) {
  const int m = n - 1;
  const long N = (long)m * m;
  double acc[2 * JMAX];
#pragma unroll
  for (int q = 0; q < 2 * JMAX; ++q) acc[q] = 0;
  for (long t = blockIdx.x * 256L + threadIdx.x; t < N; t += (long)gridDim.x * 256) {
    int k, j;
    node_of(t, m, k, j);
    const size_t idx = (size_t)k * pitch + j;
    double2 y = Y[idx];
#pragma unroll
    for (int q = 0; q < JMAX; ++q) {
      if (q < J) {
        double2 w = W[q * stride + idx];
        acc[2 * q] += w.x * y.x + w.y * y.y;
        acc[2 * q + 1] += w.x * y.y - w.y * y.x;
      }
    }
  }
  double tot[2 * JMAX];
  block_sum<2 * JMAX>(acc, tot);
  if (threadIdx.x == 0)
    for (int q = 0; q < 2 * J; ++q) part[(size_t)blockIdx.x * 2 * J + q] = tot[q];
}

// Y -= sum_q coef_q W_q  (coef on the device, complex), then per-block
// partial ||Y||^2 into part[b].
template <int JMAX>
__global__ void __launch_bounds__(256) k_multiaxpy(int n, int pitch, size_t stride,
                                                   const double2* __restrict__ W, int J,
                                                   const double2* __restrict__ coef,
                                                   double2* __restrict__ Y,
                                                   double* __restrict__ part) {
  const int m = n - 1;
  const long N = (long)m * m;
  __shared__ double2 cf[JMAX];
  if (threadIdx.x < J) cf[threadIdx.x] = coef[threadIdx.x];
  __syncthreads();
  double acc[1] = {0};
  for (long t = blockIdx.x * 256L + threadIdx.x; t < N; t += (long)gridDim.x * 256) {
    int k, j;
    node_of(t, m, k, j);
    const size_t idx = (size_t)k * pitch + j;
    double2 y = Y[idx];
#pragma unroll
    for (int q = 0; q < JMAX; ++q) {
      if (q < J) {
        double2 w = W[q * stride + idx], c = cf[q];
        y.x -= c.x * w.x - c.y * w.y;
        y.y -= c.x * w.y + c.y * w.x;
      }
    }
    Y[idx] = y;
    acc[0] += y.x * y.x + y.y * y.y;
  }
  double tot[1];
  block_sum<1>(acc, tot);
  if (threadIdx.x == 0) part[blockIdx.x] = tot[0];
}

// u += sum_q coef_q Z_q with Z stored in precision TZ.
template <typename TZ, int JMAX>
__global__ void __launch_bounds__(256) k_update(int n, int pitch, size_t stride,
                                                const v2<TZ>* __restrict__ Z, int J,
                                                const double2* __restrict__ coef,
                                                double2* __restrict__ u) {
  const int m = n - 1;
  const long N = (long)m * m;
  __shared__ double2 cf[JMAX];
  if (threadIdx.x < J) cf[threadIdx.x] = coef[threadIdx.x];
  __syncthreads();
  for (long t = blockIdx.x * 256L + threadIdx.x; t < N; t += (long)gridDim.x * 256) {
    int k, j;
    node_of(t, m, k, j);
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
  const int m = n - 1;
  const long N = (long)m * m;
  const double sc = s ? *s : 1.0;
  for (long t = blockIdx.x * 256L + threadIdx.x; t < N; t += (long)gridDim.x * 256) {
    int k, j;
    node_of(t, m, k, j);
    v2<TI> v = in[(size_t)k * pitch_in + j];
    out[(size_t)k * pitch_out + j] = mk<TO>((TO)(sc * v.x), (TO)(sc * v.y));
  }
}

// Weighted copy for the transpose solve: out = w_j w_k in  or in / (w_j w_k).
__global__ void __launch_bounds__(256) k_weight(int n, int pitch, const double2* __restrict__ w,
                                                int divide, const double2* __restrict__ in,
                                                double2* __restrict__ out) {
  const int m = n - 1;
  const long N = (long)m * m;
  for (long t = blockIdx.x * 256L + threadIdx.x; t < N; t += (long)gridDim.x * 256) {
    int k, j;
    node_of(t, m, k, j);
    v2<double> ww = cmul(w[j], w[k]);
    v2<double> v = in[(size_t)k * pitch + j];
    out[(size_t)k * pitch + j] = divide ? cdiv(v, ww) : cmul(v, ww);
  }
}

// Sum of per-block partials in fixed order: out[q] = sum_b part[b*nq + q].
__global__ void k_sum_partials(int nb, int nq, const double* __restrict__ part, double* __restrict__ out) {
  const int q = threadIdx.x;
  if (q >= nq) return;
  double s = 0;
  for (int b = 0; b < nb; ++b) s += part[(size_t)b * nq + q];
  out[q] = s;
}

// ----------------------------------------------------------------------------
// FGMRES bookkeeping on the device (single thread).  State layout in `st`
// (doubles):  see GmresState in launch.h.
__global__ void k_gmres_coef(GmresState st, int j, int pass) {
  // after a multi-dot over W_0..W_j: c_i -> h_i += s_i c_i ; axpy coefficient s_i^2 c_i
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int i = 0; i <= j; ++i) {
    double s = st.scale[i];
    double cr = st.dots[2 * i], ci = st.dots[2 * i + 1];
    if (pass == 0) { st.hcol[2 * i] = 0; st.hcol[2 * i + 1] = 0; }
    st.hcol[2 * i] += s * cr;
    st.hcol[2 * i + 1] += s * ci;
    st.axcoef[i] = make_double2(s * s * cr, s * s * ci);
  }
}

__global__ void k_gmres_step(GmresState st, int j, int m, double tol_abs) {
  // after the final norm: nrm = sqrt(st.nrm2[0]); column j of H, Givens, residual estimate
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int R = m + 1;
  double nrm = sqrt(st.nrm2[0]);
  const double sj = 1.0;   // z_j = P(v_j) with the normalised v_j
  double* H = st.H;                       // column-major (m+1) x m complex
  for (int i = 0; i <= j; ++i) {
    H[2 * (j * R + i)] = sj * st.hcol[2 * i];
    H[2 * (j * R + i) + 1] = sj * st.hcol[2 * i + 1];
  }
  H[2 * (j * R + j + 1)] = sj * nrm;
  H[2 * (j * R + j + 1) + 1] = 0;
  st.scale[j + 1] = nrm > 0 ? 1.0 / nrm : 0.0;
  // earlier rotations
  for (int i = 0; i < j; ++i) {
    double* x1 = &H[2 * (j * R + i)];
    double* x2 = &H[2 * (j * R + i + 1)];
    double cr = st.cs[2 * i], ci = st.cs[2 * i + 1], sr = st.sn[2 * i], si = st.sn[2 * i + 1];
    double a = x1[0], b = x1[1], c = x2[0], d = x2[1];
    // t1 = conj(cs) x1 + conj(sn) x2 ; t2 = -sn x1 + cs x2
    double t1r = cr * a + ci * b + sr * c + si * d;
    double t1i = cr * b - ci * a + sr * d - si * c;
    double t2r = -(sr * a - si * b) + (cr * c - ci * d);
    double t2i = -(sr * b + si * a) + (cr * d + ci * c);
    x1[0] = t1r; x1[1] = t1i; x2[0] = t2r; x2[1] = t2i;
  }
  double* hj = &H[2 * (j * R + j)];
  double* hn = &H[2 * (j * R + j + 1)];
  double den = sqrt(hj[0] * hj[0] + hj[1] * hj[1] + hn[0] * hn[0] + hn[1] * hn[1]);
  double cr = hj[0] / den, ci = hj[1] / den, sr = hn[0] / den, si = hn[1] / den;
  st.cs[2 * j] = cr; st.cs[2 * j + 1] = ci; st.sn[2 * j] = sr; st.sn[2 * j + 1] = si;
  hj[0] = den; hj[1] = 0; hn[0] = 0; hn[1] = 0;
  double gr = st.g[2 * j], gi = st.g[2 * j + 1];
  // g_{j+1} = -sn g_j ; g_j = conj(cs) g_j
  st.g[2 * (j + 1)] = -(sr * gr - si * gi);
  st.g[2 * (j + 1) + 1] = -(sr * gi + si * gr);
  st.g[2 * j] = cr * gr + ci * gi;
  st.g[2 * j + 1] = cr * gi - ci * gr;
  double est = sqrt(st.g[2 * (j + 1)] * st.g[2 * (j + 1)] + st.g[2 * (j + 1) + 1] * st.g[2 * (j + 1) + 1]);
  st.est[j] = est;
  if (st.kstar[0] < 0 && (est <= tol_abs || !(nrm > 0))) st.kstar[0] = j + 1;
}

__global__ void k_gmres_begin(GmresState st, int m) {
  // start of a restart cycle: beta = sqrt(nrm2), scale_0 = 1/beta, g = (beta, 0, ...)
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double beta = sqrt(st.nrm2[0]);
  st.scale[0] = beta > 0 ? 1.0 / beta : 0.0;
  for (int i = 0; i <= m; ++i) { st.g[2 * i] = 0; st.g[2 * i + 1] = 0; }
  st.g[0] = beta;
  st.kstar[0] = -1;
  st.beta[0] = beta;
}

__global__ void k_gmres_solve(GmresState st, int m, int mm) {
  // y = H(1:k,1:k)^{-1} g(1:k); k = first step meeting the tolerance, else the
  // mm <= m steps this cycle performed; update coefficients y_i
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int R = m + 1;
  int k = (st.kstar[0] > 0 && st.kstar[0] <= mm) ? st.kstar[0] : mm;
  st.kused[0] = k;
  double* H = st.H;
  for (int i = k - 1; i >= 0; --i) {
    double vr = st.g[2 * i], vi = st.g[2 * i + 1];
    for (int c = i + 1; c < k; ++c) {
      double hr = H[2 * (c * R + i)], hi = H[2 * (c * R + i) + 1];
      double yr = st.y[2 * c], yi = st.y[2 * c + 1];
      vr -= hr * yr - hi * yi;
      vi -= hr * yi + hi * yr;
    }
    double dr = H[2 * (i * R + i)], di = H[2 * (i * R + i) + 1];
    double den = dr * dr + di * di;
    st.y[2 * i] = (vr * dr + vi * di) / den;
    st.y[2 * i + 1] = (vi * dr - vr * di) / den;
  }
  for (int i = 0; i < m; ++i)
    st.upcoef[i] = (i < k) ? make_double2(st.y[2 * i], st.y[2 * i + 1]) : make_double2(0, 0);
}

// Iterative refinement scale: s = sqrt(N)/||r|| (RMS normalisation); sc[1] = 1/s.
__global__ void k_ir_scale(const double* nrm2, double Nn, double* sc) {
  double r = sqrt(nrm2[0]);
  double s = r > 0 ? sqrt(Nn) / r : 1.0;
  sc[0] = s;
  sc[1] = 1.0 / s;
  sc[2] = 0.0;
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
  const int m = n - 1;
  const long N = (long)m * m;
  const double pref = 2.0 * Z1 * sqrt(Z1);
  for (long t = blockIdx.x * 256L + threadIdx.x; t < N; t += (long)gridDim.x * 256) {
    int k, j;
    node_of(t, m, k, j);
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
  const long N = (long)j0 * j0;
  double acc[2] = {0, 0};
  for (long t = blockIdx.x * 256L + threadIdx.x; t < N; t += (long)gridDim.x * 256) {
    const int k = (int)(t / j0) + 1, j = (int)(t % j0) + 1;
    if (k >= n || j >= n) continue;
    const size_t idx = (size_t)k * pitch + j;
    v2<double> v12 = tm[j > k ? j : k];
    v2<double> src = csub(chi[idx], cmul(v12, u[idx]));
    const double wgt = f1[j] * f2[k];
    acc[0] += wgt * src.x;
    acc[1] += wgt * src.y;
  }
  double tot[2];
  block_sum<2>(acc, tot);
  if (threadIdx.x == 0) { part[2 * blockIdx.x] = tot[0]; part[2 * blockIdx.x + 1] = tot[1]; }
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
                    int mode, double* part) {
  hipLaunchKernelGGL((k_stencil<T, TU, TF, TO>), stencil_grid(L.n), dim3(SX, SY), 0, s, L,
                     (const v2<TU>*)u, (const v2<TF>*)f, (v2<TO>*)out, mode, part);
}
template void launch_stencil<double, double, double, double>(hipStream_t, const Level<double>&, const void*, const void*, void*, int, double*);
template void launch_stencil<double, float, double, double>(hipStream_t, const Level<double>&, const void*, const void*, void*, int, double*);
template void launch_stencil<float, float, float, float>(hipStream_t, const Level<float>&, const void*, const void*, void*, int, double*);

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
                    void* fc, int pitch_c) {
  const int nc = L.n / 2;
  dim3 grid((nc - 1 + S1CX - 1) / S1CX, (nc - 1 + S1CY - 1) / S1CY);
  hipLaunchKernelGGL((k_s1_zero<T>), grid, dim3(64, 4), 0, s, L, (const v2<T>*)f, fs, (T)omega,
                     (v2<T>*)fc, pitch_c);
}
template <typename T>
void launch_s2_zero(hipStream_t s, const Level<T>& L, const void* f, const double* fs, double omega,
                    const void* ec, int pitch_c, void* u) {
  dim3 grid((L.n - 1 + S2TX - 1) / S2TX, (L.n - 1 + S2TY - 1) / S2TY);
  hipLaunchKernelGGL((k_s2_zero<T>), grid, dim3(64, 4), 0, s, L, (const v2<T>*)f, fs, (T)omega,
                     (const v2<T>*)ec, pitch_c, (v2<T>*)u);
}

#define MGC_INST_LEVEL(T)                                                                      \
  template void launch_jacobi<T>(hipStream_t, const Level<T>&, const void*, const void*, void*, double); \
  template void launch_resid_restrict<T>(hipStream_t, const Level<T>&, const void*, const void*, void*, int); \
  template void launch_prolong_add<T>(hipStream_t, int, int, void*, const void*, int);        \
  template void launch_coarse_solve<T>(hipStream_t, const double2*, int, int, const void*, void*); \
  template void launch_s1_zero<T>(hipStream_t, const Level<T>&, const void*, const double*, double, void*, int); \
  template void launch_s2_zero<T>(hipStream_t, const Level<T>&, const void*, const double*, double, const void*, int, void*);
MGC_INST_LEVEL(double)
MGC_INST_LEVEL(float)

template <typename T>
void launch_cccs(hipStream_t s, const Level<T>& L, void* u, const void* f, const double* fs,
                 const ChanTab<T>& ch, const ChanSys<T>& SA, const ChanSys<T>& SB,
                 const CccsScratch& w) {
  const int n = L.n, pitch = L.pitch;
  const int MC = ch.M > ch.L ? ch.M : ch.L;
  v2<T>* rbuf = (v2<T>*)w.rbuf;
  v2<T>* rhoA = (v2<T>*)w.rhoA;
  v2<T>* rhoB = (v2<T>*)w.rhoB;
  v2<T>* partB = (v2<T>*)w.partB;
  v2<T>* coef = (v2<T>*)w.coef;
  v2<T>* gA = (v2<T>*)w.gA;
  v2<T>* gB = (v2<T>*)w.gB;
  v2<T>* YA = (v2<T>*)w.YA;
  v2<T>* YB = (v2<T>*)w.YB;
  v2<T>* eA = (v2<T>*)w.eA;
  v2<T>* eB = (v2<T>*)w.eB;
#define MGC_CC_DISPATCH(KERNEL, GRID, BLOCK, ...)                                   \
  if (MC <= 4) hipLaunchKernelGGL((KERNEL<T, 4>), GRID, BLOCK, 0, s, __VA_ARGS__);   \
  else if (MC <= 8) hipLaunchKernelGGL((KERNEL<T, 8>), GRID, BLOCK, 0, s, __VA_ARGS__); \
  else hipLaunchKernelGGL((KERNEL<T, 16>), GRID, BLOCK, 0, s, __VA_ARGS__);
  MGC_CC_DISPATCH(k_cccs_resid_rhoA, dim3(n - 1), dim3(64), L, (const v2<T>*)u, (const v2<T>*)f,
                  fs, rbuf, ch, rhoA);
  const int nchunks = (n - 1 + CHR - 1) / CHR;
  MGC_CC_DISPATCH(k_cccs_rhoB_part, dim3((n - 1 + 63) / 64, nchunks), dim3(64), n, pitch,
                  (const v2<T>*)rbuf, ch, partB);
  hipLaunchKernelGGL((k_cccs_rhoB_sum<T>), dim3(((n - 1) * ch.L + 255) / 256), dim3(256), 0, s, n,
                     nchunks, ch.L, (const v2<T>*)partB, rhoB);
  hipLaunchKernelGGL((k_cccs_coef<T>), dim3(1), dim3(256), 0, s, n, ch, (const v2<T>*)rhoA, coef);
  const int P = SA.P > SB.P ? SA.P : SB.P;
  hipLaunchKernelGGL((k_cccs_local<T>), dim3(P, 2), dim3(64), 0, s, SA, SB, ch, n,
                     (const v2<T>*)rhoA, (const v2<T>*)rhoB, (const v2<T>*)coef, gA, gB);
  hipLaunchKernelGGL((k_cccs_iface<T>), dim3(2), dim3(64), 0, s, SA, SB, (const v2<T>*)gA,
                     (const v2<T>*)gB, YA, YB);
  const int NM = (SA.N * SA.M > SB.N * SB.M) ? SA.N * SA.M : SB.N * SB.M;
  hipLaunchKernelGGL((k_cccs_retrieve<T>), dim3((NM + 255) / 256, 2), dim3(256), 0, s, SA, SB,
                     (const v2<T>*)gA, (const v2<T>*)gB, (const v2<T>*)YA, (const v2<T>*)YB, eA, eB);
  MGC_CC_DISPATCH(k_cccs_expand, stencil_grid(n), dim3(SX, SY), n, pitch, (v2<T>*)u, ch,
                  (const v2<T>*)eA, (const v2<T>*)eB);
#undef MGC_CC_DISPATCH
}
template void launch_cccs<double>(hipStream_t, const Level<double>&, void*, const void*, const double*,
                                  const ChanTab<double>&, const ChanSys<double>&, const ChanSys<double>&,
                                  const CccsScratch&);
template void launch_cccs<float>(hipStream_t, const Level<float>&, void*, const void*, const double*,
                                 const ChanTab<float>&, const ChanSys<float>&, const ChanSys<float>&,
                                 const CccsScratch&);

static inline int vec_blocks(int n) {
  long N = (long)(n - 1) * (n - 1);
  long b = (N + 255) / 256;
  return (int)(b < VEC_BLOCKS ? b : VEC_BLOCKS);
}
int launch_vec_blocks(int n) { return vec_blocks(n); }

void launch_multidot(hipStream_t s, int n, int pitch, size_t stride, const double2* W, int J,
                     const double2* Y, double* part) {
  const int nb = vec_blocks(n);
  if (J <= 8) hipLaunchKernelGGL((k_multidot<8>), dim3(nb), dim3(256), 0, s, n, pitch, stride, W, J, Y, part);
  else if (J <= 16) hipLaunchKernelGGL((k_multidot<16>), dim3(nb), dim3(256), 0, s, n, pitch, stride, W, J, Y, part);
  else hipLaunchKernelGGL((k_multidot<32>), dim3(nb), dim3(256), 0, s, n, pitch, stride, W, J, Y, part);
}
void launch_multiaxpy(hipStream_t s, int n, int pitch, size_t stride, const double2* W, int J,
                      const double2* coef, double2* Y, double* part) {
  const int nb = vec_blocks(n);
  if (J <= 8) hipLaunchKernelGGL((k_multiaxpy<8>), dim3(nb), dim3(256), 0, s, n, pitch, stride, W, J, coef, Y, part);
  else if (J <= 16) hipLaunchKernelGGL((k_multiaxpy<16>), dim3(nb), dim3(256), 0, s, n, pitch, stride, W, J, coef, Y, part);
  else hipLaunchKernelGGL((k_multiaxpy<32>), dim3(nb), dim3(256), 0, s, n, pitch, stride, W, J, coef, Y, part);
}
template <typename TZ>
void launch_update(hipStream_t s, int n, int pitch, size_t stride, const void* Z, int J,
                   const double2* coef, double2* u) {
  hipLaunchKernelGGL((k_update<TZ, 32>), dim3(vec_blocks(n)), dim3(256), 0, s, n, pitch, stride,
                     (const v2<TZ>*)Z, J, coef, u);
}
template void launch_update<double>(hipStream_t, int, int, size_t, const void*, int, const double2*, double2*);
template void launch_update<float>(hipStream_t, int, int, size_t, const void*, int, const double2*, double2*);

template <typename TI, typename TO>
void launch_scale_copy(hipStream_t s, int n, int pitch_in, int pitch_out, const void* in,
                       const double* sc, void* out) {
  hipLaunchKernelGGL((k_scale_copy<TI, TO>), dim3(vec_blocks(n)), dim3(256), 0, s, n, pitch_in,
                     pitch_out, (const v2<TI>*)in, sc, (v2<TO>*)out);
}
template void launch_scale_copy<double, double>(hipStream_t, int, int, int, const void*, const double*, void*);
template void launch_scale_copy<double, float>(hipStream_t, int, int, int, const void*, const double*, void*);
template void launch_scale_copy<float, double>(hipStream_t, int, int, int, const void*, const double*, void*);
template void launch_scale_copy<float, float>(hipStream_t, int, int, int, const void*, const double*, void*);

void launch_weight(hipStream_t s, int n, int pitch, const double2* w, int divide, const double2* in,
                   double2* out) {
  hipLaunchKernelGGL(k_weight, dim3(vec_blocks(n)), dim3(256), 0, s, n, pitch, w, divide, in, out);
}
void launch_sum_partials(hipStream_t s, int nb, int nq, const double* part, double* out) {
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(64), 0, s, nb, nq, part, out);
}
void launch_gmres_coef(hipStream_t s, const GmresState& st, int j, int pass) {
  hipLaunchKernelGGL(k_gmres_coef, dim3(1), dim3(1), 0, s, st, j, pass);
}
void launch_gmres_step(hipStream_t s, const GmresState& st, int j, int m, double tol_abs) {
  hipLaunchKernelGGL(k_gmres_step, dim3(1), dim3(1), 0, s, st, j, m, tol_abs);
}
void launch_gmres_begin(hipStream_t s, const GmresState& st, int m) {
  hipLaunchKernelGGL(k_gmres_begin, dim3(1), dim3(1), 0, s, st, m);
}
void launch_gmres_solve(hipStream_t s, const GmresState& st, int m, int mm) {
  hipLaunchKernelGGL(k_gmres_solve, dim3(1), dim3(1), 0, s, st, m, mm);
}
void launch_ir_scale(hipStream_t s, const double* nrm2, double Nn, double* sc) {
  hipLaunchKernelGGL(k_ir_scale, dim3(1), dim3(1), 0, s, nrm2, Nn, sc);
}
void launch_copy_scalar(hipStream_t s, const double* src, double* dst) {
  hipLaunchKernelGGL(k_copy_scalar, dim3(1), dim3(1), 0, s, src, dst);
}
void launch_fill_zero(hipStream_t s, void* p, size_t bytes) {
  hipLaunchKernelGGL(k_fill_zero, dim3(256), dim3(256), 0, s, bytes / 16, (double2*)p);
}
void launch_rhs_tp(hipStream_t s, int n, int pitch, int j0, const double2* z, double Z1, double Z2,
                   double lam, double k0, double2* chi) {
  hipLaunchKernelGGL(k_rhs_tp, dim3(vec_blocks(n)), dim3(256), 0, s, n, pitch, j0, z, Z1, Z2, lam, k0, chi);
}
void launch_zeta_part(hipStream_t s, int n, int pitch, int j0, const double2* tm, const double* f1,
                      const double* f2, const double2* u, const double2* chi, double* part) {
  hipLaunchKernelGGL(k_zeta_part, dim3(VEC_BLOCKS), dim3(256), 0, s, n, pitch, j0, tm, f1, f2, u, chi, part);
}

}  // namespace mgc
