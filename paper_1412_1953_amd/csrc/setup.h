// Host-side FP64 setup of the MG-CCCS solver: 1D grid tables, bound states,
// channel potentials, factorised channel systems and the coarsest-level
// inverse.  Everything here runs once per set_potential / set_energy; none of
// it is on the per-cycle path.
#pragma once
#include <complex>
#include <string>
#include <vector>

namespace mgc {

using cd = std::complex<double>;

// One coordinate axis on one multigrid level.
// Nodes x_j = j h, complex nodes z_j: z = x e^{i gamma} for x <= R0 (gamma = 0:
// real interior), z = R0 e^{i gamma} + (x - R0) e^{i theta} beyond (ECS,
// Sec. 2.5 / Sec. 3.3).  3-point coefficients of -1/2 d^2/dz^2 on the
// non-uniform complex grid (Sec. 2.5 eq. discrete_schrodinger):
//   a_j = -1/(2 w_j h_{j-1}), c_j = -1/(2 w_j h_j), b_j = (1/h_{j-1}+1/h_j)/(2 w_j),
//   h_j = z_{j+1} - z_j, w_j = (h_{j-1} + h_j)/2.   Index 0 and n hold zeros.
struct Axis {
  int n = 0, j0 = 0;
  double L = 0, R0 = 0, theta = 0, gamma = 0, h = 0;
  std::vector<cd> z, hs, w, a, b, c;
};
Axis make_axis(int n, double L, double R0, double theta, double gamma);

// Pivoted LU of a general complex tridiagonal matrix (sub, diag, super).
struct TriLU {
  int m = 0;
  std::vector<cd> l, d, u1, u2;
  std::vector<int> swapped;
  bool factor(const std::vector<cd>& sub, const std::vector<cd>& diag,
              const std::vector<cd>& super);
  void solve(std::vector<cd>& x) const;
};

// Eigenvalues of a complex-symmetric tridiagonal matrix (diag d, off-diag e).
bool cs_tridiag_eigenvalues(std::vector<cd> d, std::vector<cd> e, std::vector<cd>& out,
                            std::string& err);

// Lowest-M bound states of H = -1/2 d^2/dz^2 + V on an axis (interior nodes).
// lam[M], phi[M][n+1] (zero on the ring), bilinear normalisation
// sum_j w_j phi_j^2 = 1, sign: entry of largest modulus has Re > 0.
bool bound_states(const Axis& ax, const std::vector<cd>& V, int M, int refine_steps,
                  std::vector<cd>& lam, std::vector<std::vector<cd>>& phi, std::string& err);

// Dense complex LU with partial pivoting; inverse written row-major.
bool dense_inverse(int N, std::vector<cd> A, std::vector<cd>& inv, std::string& err);

// Partitioned (SPIKE-type) factorisation of the block-tridiagonal channel
// system   a_t e_{t-1} + D_t e_t + c_t e_{t+1} = r_t,  t = 1..N (N = n-1),
// with scalar off-diagonal couplings and dense MxM diagonal blocks D_t.
// Rows are split into P chunks; every chunk is factorised by block LU, the
// chunk couplings are resolved through a block-tridiagonal interface system of
// (P-1) rows of 2M x 2M blocks.
struct ChannelFactors {
  int N = 0, M = 0, P = 0;
  std::vector<int> start;          // P+1 chunk boundaries (0-based rows)
  std::vector<cd> G;               // [N][M][M]  inverse local Schur complements
  std::vector<cd> lo, up;          // [N] a_t, c_t
  std::vector<cd> Vs, Ws;          // [N][M][M]  right / left spikes
  // interface system, block Thomas factors for q = 0..P-2:
  std::vector<cd> Rinv;            // [P-1][2M][2M]  inverse Schur blocks
  std::vector<cd> Rlo, Rup;        // [P-1][2M][2M]  sub / super blocks
  // the interface solve as one matrix: Y = Tif h for h_q = Rinv_q rhs_q
  // (both sweeps applied to unit vectors), [(P-1)2M][(P-1)2M] row-major
  std::vector<cd> Tif;
};
bool factor_channels(int N, int M, int P, const std::vector<cd>& lo,
                     const std::vector<cd>& up, const std::vector<cd>& D,
                     ChannelFactors& out, std::string& err);
// Reference solve with the factors (host, used for self-checks).
void solve_channels_host(const ChannelFactors& f, std::vector<cd>& rhs);

}  // namespace mgc
