// Host-side FP64 setup: grid tables, 1D bound states, channel factors,
// coarsest-level inverse.  See setup.h.
#include "setup.h"

#include <algorithm>
#include <cmath>
#include <numeric>

namespace mgc {

static inline double cabs1(cd v) { return std::abs(v.real()) + std::abs(v.imag()); }

Axis make_axis(int n, double L, double R0, double theta, double gamma) {
  Axis ax;
  ax.n = n; ax.L = L; ax.R0 = R0; ax.theta = theta; ax.gamma = gamma;
  ax.h = L / n;
  ax.j0 = (int)std::lround(R0 / ax.h);
  const cd rot_in = std::polar(1.0, gamma), rot_out = std::polar(1.0, theta);
  ax.z.assign(n + 1, 0.0);
  for (int j = 0; j <= n; ++j) {
    double x = j * ax.h;
    ax.z[j] = (j <= ax.j0) ? x * rot_in : R0 * rot_in + (x - R0) * rot_out;
  }
  ax.hs.assign(n, 0.0);
  for (int j = 0; j < n; ++j) ax.hs[j] = ax.z[j + 1] - ax.z[j];
  ax.w.assign(n + 1, 0.0); ax.a = ax.w; ax.b = ax.w; ax.c = ax.w;
  for (int j = 1; j < n; ++j) {
    cd hm = ax.hs[j - 1], hp = ax.hs[j];
    cd w = 0.5 * (hm + hp);
    ax.w[j] = w;
    ax.a[j] = -1.0 / (2.0 * w * hm);
    ax.c[j] = -1.0 / (2.0 * w * hp);
    ax.b[j] = (1.0 / hm + 1.0 / hp) / (2.0 * w);
  }
  return ax;
}

// ---------------------------------------------------------------------------
// Tridiagonal LU with adjacent-row partial pivoting.  After factoring, row i
// of U holds d[i] (diagonal), u1[i] (first super), u2[i] (second super, only
// non-zero where rows were exchanged); l[i] is the multiplier that eliminated
// the sub-diagonal entry of column i.
bool TriLU::factor(const std::vector<cd>& sub, const std::vector<cd>& diag,
                   const std::vector<cd>& super) {
  m = (int)diag.size();
  d = diag;
  u1.assign(m, 0.0); u2.assign(m, 0.0); l.assign(m, 0.0); swapped.assign(m, 0);
  for (int i = 0; i + 1 < m; ++i) u1[i] = super[i];
  std::vector<cd> s(sub);           // s[i] = entry (i+1, i)
  for (int i = 0; i + 1 < m; ++i) {
    cd below = s[i];
    if (cabs1(d[i]) >= cabs1(below)) {
      if (d[i] == 0.0) return false;
      cd mult = below / d[i];
      l[i] = mult;
      d[i + 1] -= mult * u1[i];
    } else {
      // exchange rows i and i+1, then eliminate
      cd ri0 = d[i], ri1 = u1[i];                       // old row i: (d, u1, 0)
      cd rn0 = below, rn1 = d[i + 1], rn2 = (i + 2 < m) ? u1[i + 1] : cd(0.0);
      d[i] = rn0; u1[i] = rn1; u2[i] = rn2;
      cd mult = ri0 / rn0;
      l[i] = mult;
      swapped[i] = 1;
      d[i + 1] = ri1 - mult * rn1;
      if (i + 2 < m) u1[i + 1] = -mult * rn2;
    }
  }
  return d[m - 1] != 0.0;
}

void TriLU::solve(std::vector<cd>& x) const {
  for (int i = 0; i + 1 < m; ++i) {
    if (swapped[i]) std::swap(x[i], x[i + 1]);
    x[i + 1] -= l[i] * x[i];
  }
  for (int i = m - 1; i >= 0; --i) {
    cd v = x[i];
    if (i + 1 < m) v -= u1[i] * x[i + 1];
    if (i + 2 < m) v -= u2[i] * x[i + 2];
    x[i] = v / d[i];
  }
}

// ---------------------------------------------------------------------------
// Implicit QL iteration with a Wilkinson-type shift on a complex-symmetric
// tridiagonal matrix.  The plane rotations are complex orthogonal
// (c^2 + s^2 = 1) so the matrix stays complex symmetric; eigenvalues converge
// at the top of each unreduced block and are deflated there.
bool cs_tridiag_eigenvalues(std::vector<cd> d, std::vector<cd> e, std::vector<cd>& out,
                            std::string& err) {
  const int m = (int)d.size();
  e.resize(m, 0.0);
  e[m - 1] = 0.0;
  const double eps = 2.220446049250313e-16;
  for (int top = 0; top < m; ++top) {
    int sweeps = 0;
    for (;;) {
      int bot = top;
      for (; bot < m - 1; ++bot) {
        double scale = cabs1(d[bot]) + cabs1(d[bot + 1]);
        if (cabs1(e[bot]) <= eps * scale) break;
      }
      if (bot == top) break;
      if (++sweeps > 200) { err = "QL iteration did not converge"; return false; }
      // shift: eigenvalue of the leading 2x2 block closest to d[top]
      cd q = (d[top + 1] - d[top]) / (2.0 * e[top]);
      cd rad = std::sqrt(q * q + 1.0);
      cd den = (std::abs(q + rad) >= std::abs(q - rad)) ? q + rad : q - rad;
      cd shift = d[top] - e[top] / den;
      // chase from the bottom of the block to the top
      cd g = d[bot] - shift, s = 1.0, c = 1.0, p = 0.0;
      bool early = false;
      for (int i = bot - 1; i >= top; --i) {
        cd f = s * e[i], b = c * e[i];
        cd r = std::sqrt(f * f + g * g);
        e[i + 1] = r;
        if (std::abs(r) == 0.0) {
          d[i + 1] -= p;
          e[bot] = 0.0;
          early = true;
          break;
        }
        s = f / r;
        c = g / r;
        cd gg = d[i + 1] - p;
        cd t = (d[i] - gg) * s + 2.0 * c * b;
        p = s * t;
        d[i + 1] = gg + p;
        g = c * t - b;
      }
      if (early) continue;
      d[top] -= p;
      e[top] = g;
      e[bot] = 0.0;
    }
  }
  out = d;
  return true;
}

// Lowest-M selection: smallest real part, near ties (|dRe| < 1e-12) to the
// smaller |Im|.
static std::vector<int> select_lowest(const std::vector<cd>& ev, int M) {
  std::vector<int> order(ev.size());
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(),
                   [&](int x, int y) { return ev[x].real() < ev[y].real(); });
  std::vector<int> out;
  size_t i = 0;
  while (i < order.size() && (int)out.size() < M) {
    size_t j = i + 1;
    while (j < order.size() && std::abs(ev[order[j]].real() - ev[order[i]].real()) < 1e-12) ++j;
    std::vector<int> grp(order.begin() + i, order.begin() + j);
    std::stable_sort(grp.begin(), grp.end(), [&](int x, int y) {
      return std::abs(ev[x].imag()) < std::abs(ev[y].imag());
    });
    out.insert(out.end(), grp.begin(), grp.end());
    i = j;
  }
  out.resize(M);
  return out;
}

bool bound_states(const Axis& ax, const std::vector<cd>& V, int M, int refine_steps,
                  std::vector<cd>& lam, std::vector<std::vector<cd>>& phi, std::string& err) {
  const int n = ax.n, m = n - 1;
  lam.assign(M, 0.0);
  phi.assign(M, std::vector<cd>(n + 1, 0.0));
  if (M == 0) return true;
  // Symmetrised standard form T = W^{-1/2} S W^{-1/2} of S phi = lam W phi,
  // S = W H (complex symmetric), same spectrum.
  std::vector<cd> sw(n + 1, 0.0), dT(m), eT(m, 0.0);
  for (int j = 1; j < n; ++j) sw[j] = std::sqrt(ax.w[j]);
  for (int j = 1; j < n; ++j) dT[j - 1] = ax.b[j] + V[j];
  for (int j = 1; j + 1 < n; ++j)  // S_{j,j+1} = w_j c_j = -1/(2 h_j)
    eT[j - 1] = (ax.w[j] * ax.c[j]) / (sw[j] * sw[j + 1]);
  std::vector<cd> ev;
  if (!cs_tridiag_eigenvalues(dT, eT, ev, err)) return false;
  std::vector<int> sel = select_lowest(ev, M);

  // S - sigma W as a tridiagonal matrix on interior nodes 1..n-1
  std::vector<cd> Sd(m), Ss(m, 0.0), Sp(m, 0.0), wv(m);
  for (int j = 1; j < n; ++j) {
    Sd[j - 1] = ax.w[j] * (ax.b[j] + V[j]);
    wv[j - 1] = ax.w[j];
  }
  for (int j = 1; j + 1 < n; ++j) { Sp[j - 1] = ax.w[j] * ax.c[j]; Ss[j - 1] = ax.w[j + 1] * ax.a[j + 1]; }
  auto bilinear_normalise = [&](std::vector<cd>& v) {
    cd s = 0.0;
    for (int t = 0; t < m; ++t) s += wv[t] * v[t] * v[t];
    cd nrm = std::sqrt(s);
    for (auto& x : v) x /= nrm;
  };
  for (int k = 0; k < M; ++k) {
    cd sigma = ev[sel[k]];
    // inverse iteration from the QL eigenvalue: 3 steps to converge the
    // vector, then the shift-and-invert refinement steps of Sec. 5.1.
    std::vector<cd> diag(m);
    for (int t = 0; t < m; ++t) diag[t] = Sd[t] - sigma * wv[t];
    TriLU lu;
    if (!lu.factor(Ss, diag, Sp)) {
      // exact singularity: nudge the shift by one ulp-scale amount
      sigma += cd(1e-14 * (1.0 + std::abs(sigma)), 0.0);
      for (int t = 0; t < m; ++t) diag[t] = Sd[t] - sigma * wv[t];
      if (!lu.factor(Ss, diag, Sp)) { err = "singular shifted operator"; return false; }
    }
    std::vector<cd> v(m);
    for (int t = 0; t < m; ++t) v[t] = 1.0 + 0.37 * std::sin(1.0 + 0.71 * t);
    for (int it = 0; it < 3 + refine_steps; ++it) {
      for (int t = 0; t < m; ++t) v[t] *= wv[t];
      lu.solve(v);
      bilinear_normalise(v);
    }
    int imax = 0;
    for (int t = 1; t < m; ++t) if (std::abs(v[t]) > std::abs(v[imax])) imax = t;
    if (v[imax].real() < 0) for (auto& x : v) x = -x;
    // Rayleigh quotient (bilinear): v^T S v / v^T W v
    cd num = 0.0, den = 0.0;
    for (int t = 0; t < m; ++t) {
      cd Sv = Sd[t] * v[t];
      if (t > 0) Sv += Ss[t - 1] * v[t - 1];
      if (t + 1 < m) Sv += Sp[t] * v[t + 1];
      num += v[t] * Sv;
      den += wv[t] * v[t] * v[t];
    }
    lam[k] = num / den;
    for (int t = 0; t < m; ++t) phi[k][t + 1] = v[t];
  }
  return true;
}

// ---------------------------------------------------------------------------
static bool lu_inplace(int N, std::vector<cd>& A, std::vector<int>& piv) {
  piv.resize(N);
  for (int k = 0; k < N; ++k) {
    int p = k;
    double best = std::abs(A[(size_t)k * N + k]);
    for (int i = k + 1; i < N; ++i) {
      double v = std::abs(A[(size_t)i * N + k]);
      if (v > best) { best = v; p = i; }
    }
    if (best == 0.0) return false;
    piv[k] = p;
    if (p != k)
      for (int j = 0; j < N; ++j) std::swap(A[(size_t)k * N + j], A[(size_t)p * N + j]);
    cd inv = 1.0 / A[(size_t)k * N + k];
    for (int i = k + 1; i < N; ++i) {
      cd f = A[(size_t)i * N + k] * inv;
      A[(size_t)i * N + k] = f;
      if (f == 0.0) continue;
      for (int j = k + 1; j < N; ++j) A[(size_t)i * N + j] -= f * A[(size_t)k * N + j];
    }
  }
  return true;
}

static void lu_solve_vec(int N, const std::vector<cd>& LU, const std::vector<int>& piv,
                         cd* x) {
  for (int k = 0; k < N; ++k) if (piv[k] != k) std::swap(x[k], x[piv[k]]);
  for (int i = 0; i < N; ++i) {
    cd s = x[i];
    for (int j = 0; j < i; ++j) s -= LU[(size_t)i * N + j] * x[j];
    x[i] = s;
  }
  for (int i = N - 1; i >= 0; --i) {
    cd s = x[i];
    for (int j = i + 1; j < N; ++j) s -= LU[(size_t)i * N + j] * x[j];
    x[i] = s / LU[(size_t)i * N + i];
  }
}

bool dense_inverse(int N, std::vector<cd> A, std::vector<cd>& inv, std::string& err) {
  std::vector<int> piv;
  if (!lu_inplace(N, A, piv)) { err = "singular dense matrix"; return false; }
  inv.assign((size_t)N * N, 0.0);
  std::vector<cd> col(N);
  for (int j = 0; j < N; ++j) {
    std::fill(col.begin(), col.end(), 0.0);
    col[j] = 1.0;
    lu_solve_vec(N, A, piv, col.data());
    for (int i = 0; i < N; ++i) inv[(size_t)i * N + j] = col[i];
  }
  return true;
}

// ---------------------------------------------------------------------------
// small dense helpers on row-major R x R blocks
static void matmul(int R, const cd* X, const cd* Y, cd* Z) {
  for (int i = 0; i < R; ++i)
    for (int j = 0; j < R; ++j) {
      cd s = 0.0;
      for (int k = 0; k < R; ++k) s += X[i * R + k] * Y[k * R + j];
      Z[i * R + j] = s;
    }
}
static void matvec(int R, const cd* X, const cd* v, cd* out) {
  for (int i = 0; i < R; ++i) {
    cd s = 0.0;
    for (int k = 0; k < R; ++k) s += X[i * R + k] * v[k];
    out[i] = s;
  }
}

bool factor_channels(int N, int M, int P, const std::vector<cd>& lo,
                     const std::vector<cd>& up, const std::vector<cd>& D,
                     ChannelFactors& f, std::string& err) {
  f = ChannelFactors();
  f.N = N; f.M = M; f.P = P; f.lo = lo; f.up = up;
  const size_t MM = (size_t)M * M;
  f.start.resize(P + 1);
  for (int p = 0; p <= P; ++p) f.start[p] = (int)(((long long)N * p) / P);
  for (int p = 0; p < P; ++p)
    if (f.start[p + 1] - f.start[p] < 1) { err = "empty channel chunk"; return false; }
  f.G.assign(N * MM, 0.0);
  f.Vs.assign(N * MM, 0.0);
  f.Ws.assign(N * MM, 0.0);
  std::vector<cd> tmp(MM), tmp2(MM);
  // local block LU per chunk
  for (int p = 0; p < P; ++p) {
    for (int t = f.start[p]; t < f.start[p + 1]; ++t) {
      std::vector<cd> Dp(D.begin() + t * MM, D.begin() + (t + 1) * MM);
      if (t > f.start[p]) {
        const cd s = lo[t] * up[t - 1];
        for (size_t q = 0; q < MM; ++q) Dp[q] -= s * f.G[(t - 1) * MM + q];
      }
      std::vector<cd> inv;
      if (!dense_inverse(M, Dp, inv, err)) { err = "singular channel block"; return false; }
      std::copy(inv.begin(), inv.end(), f.G.begin() + t * MM);
    }
  }
  // spikes: right V (coupling of the last chunk row to the next chunk) and
  // left W (coupling of the first chunk row to the previous chunk)
  for (int p = 0; p < P; ++p) {
    const int s = f.start[p], e = f.start[p + 1] - 1;
    if (p + 1 < P) {
      // forward: Z_e = G_e * (c_e I); backward X_t = -c_t G_t X_{t+1}
      for (size_t q = 0; q < MM; ++q) f.Vs[e * MM + q] = f.G[e * MM + q] * up[e];
      for (int t = e - 1; t >= s; --t) {
        matmul(M, &f.G[t * MM], &f.Vs[(t + 1) * MM], tmp.data());
        for (size_t q = 0; q < MM; ++q) f.Vs[t * MM + q] = -up[t] * tmp[q];
      }
    }
    if (p > 0) {
      // forward Z_s = G_s a_s, Z_t = -a_t G_t Z_{t-1}; backward X_t = Z_t - c_t G_t X_{t+1}
      for (size_t q = 0; q < MM; ++q) f.Ws[s * MM + q] = f.G[s * MM + q] * lo[s];
      for (int t = s + 1; t <= e; ++t) {
        matmul(M, &f.G[t * MM], &f.Ws[(t - 1) * MM], tmp.data());
        for (size_t q = 0; q < MM; ++q) f.Ws[t * MM + q] = -lo[t] * tmp[q];
      }
      for (int t = e - 1; t >= s; --t) {
        matmul(M, &f.G[t * MM], &f.Ws[(t + 1) * MM], tmp.data());
        for (size_t q = 0; q < MM; ++q) f.Ws[t * MM + q] -= up[t] * tmp[q];
      }
    }
  }
  // interface system: unknown Y_q = [B_q ; T_{q+1}] for q = 0..P-2
  const int Q = P - 1, R = 2 * M;
  const size_t RR = (size_t)R * R;
  f.Rinv.assign((size_t)std::max(Q, 0) * RR, 0.0);
  f.Rlo.assign(f.Rinv.size(), 0.0);
  f.Rup.assign(f.Rinv.size(), 0.0);
  std::vector<cd> Rd(RR), Sub(RR), Sup(RR), prevRinvSup(RR, 0.0), X(RR);
  for (int q = 0; q < Q; ++q) {
    const int e_q = f.start[q + 1] - 1, s_n = f.start[q + 1];
    std::fill(Rd.begin(), Rd.end(), 0.0);
    std::fill(Sub.begin(), Sub.end(), 0.0);
    std::fill(Sup.begin(), Sup.end(), 0.0);
    for (int i = 0; i < M; ++i) {
      Rd[i * R + i] = 1.0;
      Rd[(M + i) * R + (M + i)] = 1.0;
      for (int k = 0; k < M; ++k) {
        Rd[i * R + (M + k)] = f.Vs[e_q * MM + i * M + k];          // V_q[e] T_{q+1}
        Rd[(M + i) * R + k] = f.Ws[s_n * MM + i * M + k];          // W_{q+1}[s] B_q
        if (q > 0) Sub[i * R + k] = f.Ws[e_q * MM + i * M + k];    // W_q[e] B_{q-1}
        if (q + 1 < Q) Sup[(M + i) * R + (M + k)] = f.Vs[s_n * MM + i * M + k];  // V_{q+1}[s] T_{q+2}
      }
    }
    if (q > 0) {
      matmul(R, Sub.data(), prevRinvSup.data(), X.data());
      for (size_t t = 0; t < RR; ++t) Rd[t] -= X[t];
    }
    std::vector<cd> inv;
    if (!dense_inverse(R, Rd, inv, err)) { err = "singular interface block"; return false; }
    std::copy(inv.begin(), inv.end(), f.Rinv.begin() + q * RR);
    matmul(R, inv.data(), Sub.data(), &f.Rlo[q * RR]);
    matmul(R, inv.data(), Sup.data(), &f.Rup[q * RR]);
    std::copy(f.Rup.begin() + q * RR, f.Rup.begin() + (q + 1) * RR, prevRinvSup.begin());
  }
  // the two sweeps (forward Z_q = h_q - Rlo_q Z_{q-1}, backward Y_q = Z_q -
  // Rup_q Y_{q+1}) are linear in h: apply them to every unit vector
  const size_t QR = (size_t)std::max(Q, 0) * R;
  f.Tif.assign(QR * QR, 0.0);
  std::vector<cd> Y(QR), t(R);
  for (size_t c = 0; c < QR; ++c) {
    std::fill(Y.begin(), Y.end(), 0.0);
    Y[c] = 1.0;
    for (int q = 1; q < Q; ++q) {
      matvec(R, &f.Rlo[q * RR], &Y[(q - 1) * R], t.data());
      for (int i = 0; i < R; ++i) Y[q * R + i] -= t[i];
    }
    for (int q = Q - 2; q >= 0; --q) {
      matvec(R, &f.Rup[q * RR], &Y[(q + 1) * R], t.data());
      for (int i = 0; i < R; ++i) Y[q * R + i] -= t[i];
    }
    for (size_t r = 0; r < QR; ++r) f.Tif[r * QR + c] = Y[r];
  }
  return true;
}

void solve_channels_host(const ChannelFactors& f, std::vector<cd>& x) {
  const int N = f.N, M = f.M, P = f.P;
  const size_t MM = (size_t)M * M;
  std::vector<cd> g(x.size()), v(M), w(M);
  // local solves
  for (int p = 0; p < P; ++p) {
    const int s = f.start[p], e = f.start[p + 1] - 1;
    for (int t = s; t <= e; ++t) {
      for (int i = 0; i < M; ++i) v[i] = x[t * M + i] - (t > s ? f.lo[t] * g[(t - 1) * M + i] : 0.0);
      matvec(M, &f.G[t * MM], v.data(), &g[t * M]);
    }
    for (int t = e - 1; t >= s; --t) {
      matvec(M, &f.G[t * MM], &g[(t + 1) * M], w.data());
      for (int i = 0; i < M; ++i) g[t * M + i] -= f.up[t] * w[i];
    }
  }
  // interface system
  const int Q = P - 1, R = 2 * M;
  const size_t RR = (size_t)R * R;
  std::vector<cd> Z((size_t)std::max(Q, 0) * R), rhs(R), tmp(R);
  for (int q = 0; q < Q; ++q) {
    const int e_q = f.start[q + 1] - 1, s_n = f.start[q + 1];
    for (int i = 0; i < M; ++i) { rhs[i] = g[e_q * M + i]; rhs[M + i] = g[s_n * M + i]; }
    matvec(R, &f.Rinv[q * RR], rhs.data(), &Z[q * R]);
    if (q > 0) {
      matvec(R, &f.Rlo[q * RR], &Z[(q - 1) * R], tmp.data());
      for (int i = 0; i < R; ++i) Z[q * R + i] -= tmp[i];
    }
  }
  for (int q = Q - 2; q >= 0; --q) {
    matvec(R, &f.Rup[q * RR], &Z[(q + 1) * R], tmp.data());
    for (int i = 0; i < R; ++i) Z[q * R + i] -= tmp[i];
  }
  // retrieval x_t = g_t - V_t T_{p+1} - W_t B_{p-1}
  for (int p = 0; p < P; ++p) {
    const int s = f.start[p], e = f.start[p + 1] - 1;
    for (int t = s; t <= e; ++t) {
      for (int i = 0; i < M; ++i) x[t * M + i] = g[t * M + i];
      if (p + 1 < P) {
        matvec(M, &f.Vs[t * MM], &Z[p * R + M], w.data());
        for (int i = 0; i < M; ++i) x[t * M + i] -= w[i];
      }
      if (p > 0) {
        matvec(M, &f.Ws[t * MM], &Z[(p - 1) * R], w.data());
        for (int i = 0; i < M; ++i) x[t * M + i] -= w[i];
      }
    }
  }
}

}  // namespace mgc
