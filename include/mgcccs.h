/*
 * mgcccs.h -- C ABI of the MI355X (gfx950) MG-CCCS solver for the 2D driven
 * Schroedinger equation  (H - E) u = chi  on an exterior-complex-scaled grid.
 *
 * Method: Cools & Vanroose, "A fast and robust computational method for the
 * ionization cross sections of the driven Schroedinger equation using an O(N)
 * multigrid-based scheme" (arXiv:1412.1953):
 *   - problem and boundary conditions: Sec. 2.2, eq. partialwave2d;
 *   - finite-difference discretisation: Sec. 2.5, eq. discrete_schrodinger;
 *   - Temkin-Poet potentials -Z1/x, -Z2/y, lambda/max(x,y): Sec. 5.2, Sec. 6.2;
 *   - multigrid V(1,1) cycle with omega-Jacobi, full weighting and bilinear
 *     interpolation: Sec. 1 and Sec. 3.2;
 *   - Coupled Channel Correction Step (CCCS): Sec. 4, eqs. coupled_channel_expansion,
 *     convention_a/b, coefficients, channel1/channel2, cccs;
 *   - MG-CCCS as a Krylov (FGMRES) preconditioner: Sec. 6, Table 1;
 *   - ionisation amplitude and cross section: Sec. 3.3, eqs. double-ionization,
 *     testfunction, total-double-ionization.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Fields.  A field on level l is an (n_l+1) x pitch_l array of interleaved
 *   complex numbers (double2 for MGC_FP64, float2 for MGC_FP32) in device
 *   memory.  Row k runs along x2, column j along x1 (contiguous); element
 *   (k, j) lives at k*pitch_l + j.  Rows/columns 0 and n_l are the homogeneous
 *   Dirichlet ring: the library never reads or writes them (they are treated as
 *   zero).  Columns beyond n_l are padding and are never touched.  The level-0
 *   pitch is returned by mgc_field_pitch().
 * Ownership.  The caller owns every field and the workspace; the library owns
 *   only host-side setup data and never allocates device memory.  All device
 *   pointers must belong to the device that was current at mgc_create_grid.
 * Streams.  All device work is enqueued on the stream given at creation (NULL
 *   = default stream).  Calls that return host scalars (relres, zeta, stats)
 *   synchronise that stream; the others are asynchronous.
 * Errors.  Every entry point returns an mgc_status.  Arguments are validated
 *   before any side effect (MGC_EINVAL).  A HIP runtime error returns MGC_EHIP
 *   and marks the handle failed: later calls return MGC_ESTATE.  A solve that
 *   reaches max_it returns MGC_ENOCONV with u = last iterate and stats filled; a
 *   NaN/Inf residual returns MGC_ENUMERIC.  mgc_last_error() gives a message.
 * Threads.  A handle is not thread-safe; distinct handles are independent.
 */
#ifndef MGCCCS_H
#define MGCCCS_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MGC_OK = 0,
  MGC_EINVAL = -1,    /* invalid argument (nothing was changed)                */
  MGC_ENOMEM = -2,    /* bound workspace too small                             */
  MGC_EHIP = -3,      /* HIP runtime error; handle is now failed               */
  MGC_ENOCONV = -4,   /* iteration limit reached before the tolerance          */
  MGC_ESTATE = -5,    /* call order violated or handle failed                  */
  MGC_ENUMERIC = -6   /* NaN or Inf encountered                                */
} mgc_status;

/* Largest FGMRES restart length (basis size) the library supports. */
#define MGC_MAX_RESTART 16

/* Most momentum pairs one mgc_cross_section_sweep call evaluates. */
#define MGC_SWEEP_MAX 256

typedef enum { MGC_FP64 = 0, MGC_FP32 = 1 } mgc_precision;

typedef enum {
  MGC_STATIONARY = 0, /* repeat {V-cycle; CCCS} on A u = f (Sec. 6.1)          */
  MGC_IR = 1,         /* FP64 iterative refinement around inner MG-CCCS cycles */
  MGC_FGMRES = 2,     /* FP64 FGMRES(restart), right-preconditioned by one
                         MG-CCCS cycle started from zero (Sec. 6, Table 1)      */
  MGC_BICGSTAB = 3    /* FP64 BiCGSTAB right-preconditioned by one MG-CCCS cycle
                         from zero (Sec. 6.1, Fig. convrate2D): shadow vector =
                         initial residual, conjugated inner products; two
                         cycles per iteration.  Needs desc.max_restart >= 5
                         (its six vectors live in the Krylov basis).            */
} mgc_outer;

typedef struct mgc_grid_s* mgc_grid;   /* opaque, library-owned host object */

/* Grid and solver structure (fixed for the life of a handle).
 * n        intervals per dimension on the finest level; a power of two >= 8.
 * L, R0    domain [0,L]^2; complex scaling starts at x = R0, which must be a
 *          node of the coarsest level (R0/(L/n_coarsest) integral), 0 < R0 < L.
 * theta    ECS angle in (0, pi/2): z = R0 + (x - R0) e^{i theta} for x > R0.
 * levels   multigrid levels including the coarsest (n >> (levels-1) >= 4);
 *          the coarsest level is solved by a dense FP64 direct solve and must
 *          hold at most 1024 unknowns.
 * M, Lch   channels (lowest 1D eigenstates) in x1 and in x2; 0 <= M,Lch <= 16.
 *          M = Lch = 0 disables the CCCS.
 * omega, nu1, nu2   omega-Jacobi weight and pre/post smoothing sweeps.
 * pc_gamma, pc_first_level, pc_gamma0
 *          interior contour rotation used by the preconditioning hierarchy:
 *          on levels >= pc_first_level the grid is z = x e^{i pc_gamma} for
 *          x <= R0 (the complex-contour operator of Sec. 3.1/Sec. 6), followed
 *          by the ECS ray; levels below pc_first_level use the angle
 *          pc_gamma0 in the same way.  pc_gamma = pc_gamma0 = 0 makes every
 *          level the exact operator.  Both angles lie in [0, pi/4).  The
 *          CCCS acts on the level-0 operator of the hierarchy.
 * max_restart  FGMRES basis size the workspace must hold, 0 .. MGC_MAX_RESTART
 *              (0: no FGMRES; BiCGSTAB needs at least 5).
 * gamma    contour angle of the system itself, [0, pi/4): the operator A is
 *          discretised on z = x e^{i gamma} for x <= R0 followed by the ECS ray
 *          (0: the exterior-complex-scaled grid with a real interior; R0 = L
 *          with gamma > 0: the full complex contour of Sec. 3.1 / Sec. 6).
 *          The amplitude and cross-section calls need gamma = 0.
 * smoother MGC_SMOOTH_JACOBI (0): omega-Jacobi; MGC_SMOOTH_GMRES3 (1): one
 *          GMRES(3) cycle per smoothing step instead (the substitute of
 *          Sec. 6.1; u += V y minimising the level's residual over the
 *          3-dimensional Krylov space of its residual), which takes four more
 *          fields per level and runs the cycle's general (per-level) path.
 * pc_order MGC_PC_MG_CCCS (0): the Krylov preconditioner is the MG-CCCS
 *          cycle of Sec. 4.3 (V-cycle, then the channel correction of its
 *          residual); MGC_PC_DEFLATION (1): the channel correction embedded as
 *          a deflation step (the alternative named in Sec. 7): z1 = e*(v)
 *          first, then z = z1 + V(v - A z1) with one V-cycle from zero on the
 *          deflated residual.  Applies to the FGMRES and BiCGSTAB
 *          preconditioner; takes one more level-0 field per precision.
 * pot_tables 0: the two-body potential is the Temkin-Poet lambda/max(x1,x2),
 *          applied from 1D tables; 1: the workspace also holds one general
 *          two-body table per level and precision (a field of V12 at the
 *          level's nodes), which mgc_set_potential_exp requires.
 * gs_from  with MGC_SMOOTH_GMRES3: the first level that takes the GMRES(3)
 *          substitute; the levels above it (finer) keep omega-Jacobi.  0 = every
 *          level (Sec. 6.1).  Jacobi on the fine levels, where kh is small,
 *          and a Krylov smoother on the coarse ones, where Jacobi amplifies the
 *          near-resonant modes, is the split of Krylov-enhanced Helmholtz
 *          multigrid (Elman, Ernst and O'Leary, 2001).  Must lie in [0, levels].
 * precisions   bit mask (1 << MGC_FP64) | (1 << MGC_FP32) of the cycle
 *          precisions the workspace must hold.                                */
#define MGC_SMOOTH_JACOBI 0
#define MGC_SMOOTH_GMRES3 1
#define MGC_PC_MG_CCCS 0
#define MGC_PC_DEFLATION 1
typedef struct {
  int n;
  double L, R0, theta;
  int levels;
  int M, Lch;
  double omega;
  int nu1, nu2;
  double pc_gamma;
  int pc_first_level;
  int max_restart;
  int precisions;
  double pc_gamma0;
  double gamma;
  int smoother;
  int pc_order;
  int pot_tables;
  int gs_from;
} mgc_grid_desc;

typedef struct {
  mgc_outer outer;
  mgc_precision inner;   /* precision of the MG-CCCS cycles (STATIONARY: FP64 only) */
  int restart;           /* FGMRES restart length, <= desc.max_restart           */
  int max_it;            /* outer iterations (cycles for STATIONARY)             */
  int inner_cycles;      /* MG-CCCS cycles per IR step                           */
  double tol;            /* stop when ||f - A u||_2 / ||f||_2 <= tol             */
} mgc_solve_opts;

typedef struct {
  int iters;             /* outer iterations performed                           */
  int vcycles;           /* MG-CCCS cycles performed                             */
  double relres;         /* final ||f - A u||_2 / ||f||_2 (FP64, recomputed)     */
  double* hist;          /* optional caller array: true relres at the start and
                            after every outer step (FGMRES: every restart cycle) */
  int hist_cap;          /* capacity of hist                                      */
  int hist_len;          /* entries written to hist (<= hist_cap)                 */
  double t_setup_ms;     /* host time of the last set_potential + set_energy     */
  double t_solve_ms;     /* wall time of the solve (HIP events on the stream)    */
} mgc_stats;

/* Validate desc and build the host-side grid tables.  hip_stream is a
 * hipStream_t (may be NULL).  No device memory is touched.                     */
mgc_status mgc_create_grid(const mgc_grid_desc* desc, void* hip_stream, mgc_grid* out);

/* Bytes of device workspace the handle needs (all levels, both precisions in
 * desc.precisions, CCCS tables, channel factors, Krylov basis).               */
mgc_status mgc_workspace_bytes(mgc_grid g, size_t* bytes);

/* Bind caller-owned device memory (>= mgc_workspace_bytes, 256-byte aligned).
 * The library clears it on the handle's stream.                                */
mgc_status mgc_bind_workspace(mgc_grid g, void* dev_ptr, size_t bytes);

/* Row pitch (in complex elements) of level-l fields; level 0 is the caller's. */
mgc_status mgc_field_pitch(mgc_grid g, int level, int* pitch_elems);

/* Launch schedule of the zero-guess MG-CCCS cycle (the cycle inside FGMRES
 * and the first inner cycle of IR).  It changes how the work of the V-cycle
 * of Sec. 3.2 is cut into launches, never the arithmetic: every choice gives
 * the same iterate bit for bit.  The project's autotuner picks it per grid
 * size, channel count and precision.
 * small_tiles  bit l set: level l's fused smoothing passes use the small tiles
 *              (16 x 4 coarse points / 64 x 4 nodes) instead of the large
 *              ones (32 x 8 / 64 x 16); -1 (default): large tiles on levels
 *              with at least 512 of them.
 * level_pairs  1 (default): two consecutive small-tile levels above the
 *              coarse tail share one pre- and one post-smoothing launch;
 *              0: one launch per level and pass.
 * coarse_tail  1 (default): the levels with n <= 32 (at most four) and the
 *              coarsest solve run as two launches with the levels held in
 *              LDS; 0: per-level launches and a separate coarsest solve.
 * mgc_set_schedule returns MGC_EINVAL for small_tiles < -1 or a flag outside
 * {0, 1}; the new schedule applies from the next call.                        */
typedef struct {
  int small_tiles;
  int level_pairs;
  int coarse_tail;
} mgc_schedule;
mgc_status mgc_set_schedule(mgc_grid g, const mgc_schedule* s);
mgc_status mgc_get_schedule(mgc_grid g, mgc_schedule* s);

/* Temkin-Poet potential strengths: V1 = -Z1/x1, V2 = -Z2/x2,
 * V12 = lambda/max(x1,x2) (Sec. 6.2).  Computes the M (Lch) lowest 1D
 * eigenstates of H1 (H2) with the bilinear normalisation int phi^2 dz = 1
 * (Sec. 3.1 Remark 3), refined by two shift-and-invert steps (Sec. 5.1), and
 * the channel potentials (Sec. 4.2).  Invalidates the energy setup.           */
mgc_status mgc_set_potential(mgc_grid g, double Z1, double Z2, double lambda);

/* Exponential potentials (the model of Sec. 6.1 and Sec. 3.3 Fig. 4):
 *   V1 = -a1 exp(-b1 x1^2),  V2 = -a2 exp(-b2 x2^2),
 *   V12 = c12 exp(-d12 (x1 + x2)^2),
 * each evaluated at the complex nodes of every level's contour (analytic
 * continuation).  Sec. 6.1 uses a1 = a2 = 4.5, b1 = b2 = 1, c12 = 2,
 * d12 = 0.1, with the source exp(-3 (x1 + x2)^2) supplied by the caller as
 * a field.  Same setup as mgc_set_potential (bound states, channel potentials
 * summed directly over the nodes).  Needs a handle created with
 * pot_tables = 1 (MGC_EINVAL otherwise) and finite parameters with
 * b1, b2, d12 >= 0.  The amplitude entry points (mgc_cross_section,
 * mgc_cross_section_sweep, mgc_single_ionization, mgc_total_double_ionization
 * and the batched call) take this model's potentials on an ECS grid with a
 * real interior; the impact right-hand side builder and the gradient are
 * Temkin-Poet only and return MGC_EINVAL under this model.  Invalidates the
 * energy setup.                                                              */
mgc_status mgc_set_potential_exp(mgc_grid g, double a1, double b1, double a2, double b2, double c12,
                                 double d12);

/* Eigenvalues of the channel bound states the CCCS uses (Sec. 2.4
 * eq. 1d_eigenstate, on the hierarchy's level-0 axis): lamA[2 i], lamA[2 i + 1]
 * = real and imaginary part of lambda_i of H1 for i < M, lamB likewise for the
 * Lch states of H2 (either pointer may be null).  Host arrays.  MGC_ESTATE
 * before a set_potential call.                                                */
mgc_status mgc_channel_energies(mgc_grid g, double* lamA, double* lamB);

/* Total energy E.  Factorises the coupled channel systems (Sec. 4.3) and the
 * coarsest-level operators, uploads all tables.  Requires a bound workspace
 * and mgc_set_potential.                                                       */
mgc_status mgc_set_energy(mgc_grid g, double E);

/* Write the Temkin-Poet impact right-hand side into chi (level-0 field):
 * chi0 = (lambda/max(z1,z2) - Z2/z2) phi_1s(z1) sin(k0 z2) on the real region
 * x1, x2 <= R0, zero beyond, phi_1s(z) = 2 Z1^{3/2} z e^{-Z1 z},
 * k0 = sqrt(2(E + Z1^2/2)); chi = (chi0 + chi0^T)/sqrt(2).                    */
mgc_status mgc_build_rhs_tp(mgc_grid g, void* chi, mgc_precision prec);

/* r = f - A u on the level-0 interior (A = exact operator: ECS grid, rotation
 * 0).  relres (nullable, synchronising) receives ||r||_2/||f||_2.  u, f, r are
 * level-0 fields of precision prec; r may not alias u.                        */
mgc_status mgc_residual(mgc_grid g, const void* u, const void* f, void* r,
                        double* relres, mgc_precision prec);

/* One V(nu1,nu2)-cycle in place on u for A_h u = f, where A_h is the level-0
 * operator of the preconditioning hierarchy (Sec. 3.2).                       */
mgc_status mgc_vcycle(mgc_grid g, void* u, const void* f, mgc_precision prec);

/* One Coupled Channel Correction Step in place on u (Sec. 4.3, eq. cccs).     */
mgc_status mgc_cccs(mgc_grid g, void* u, const void* f, mgc_precision prec);

/* mgc_cccs for callers that cannot allocate device memory -- code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  It
 * allocates nothing, neither itself nor through a library: the CCCS scratch
 * (projection partials, channel right-hand sides and solutions, about
 * (2 ceil((n-1)/64) + 7) (n+1) M complex values for M = Lch) lives in a
 * static device array of MGC_NOALLOC_SCRATCH_BYTES that each GPU the library
 * runs on holds until the process ends.  The handle's bound workspace still
 * provides the setup data (bound states, channel factors).  The region a call
 * uses is cleared by a fill kernel on the handle's stream before use, so the
 * array's previous contents never matter; calls that overlap on one GPU (two
 * streams, two threads) share the array and race.  Same arguments, results
 * and errors as mgc_cccs, plus MGC_EINVAL when the scratch of this grid and
 * precision exceeds MGC_NOALLOC_SCRATCH_BYTES (n = 1024 with 16 channels in
 * FP64 fits) and MGC_EHIP when the array's device address cannot be taken.   */
#define MGC_NOALLOC_SCRATCH_BYTES (16u << 20)
mgc_status mgc_cccs_noalloc(mgc_grid g, void* u, const void* f, mgc_precision prec);

/* Solve A u = f (FP64 level-0 fields).  u holds the initial guess on entry and
 * the last iterate on exit.  stats may be NULL.                               */
mgc_status mgc_solve(mgc_grid g, void* u, const void* f,
                     const mgc_solve_opts* opts, mgc_stats* stats);

/* Solve A^T v = g (FP64).  With the dual weights W = diag(w_j w_k) the
 * weighted matrix W A is complex symmetric (Sec. 2.5), so A^T = W A W^{-1} and
 * v = W y with A y = W^{-1} g.  v holds the initial guess on entry.           */
mgc_status mgc_solve_transpose(mgc_grid g, void* v, const void* gvec,
                               const mgc_solve_opts* opts, mgc_stats* stats);

/* Double-ionisation amplitude (Sec. 3.3 eq. double-ionization) on the real
 * region x1, x2 <= R0 with trapezoid weights:
 *   zeta = sum_{j,k<=j0} t_j t_k phi_{k1}(x1_j) phi_{k2}(x2_k) (chi - V12 u)_{kj}
 * with phi_k the regular solution of eq. testfunction (3-point recurrence
 * with the x1 one-body potential of the model at the real nodes) normalised to
 * asymptotic amplitude 1/sqrt(k) at R0, and
 * sigma = 8 pi^2 / k0^2 * |zeta|^2 / (k1 k2), k0^2 twice the energy of the
 * incoming electron over the target's ground state: 2 E + Z1^2 for the
 * Temkin-Poet model, 2 (E - lambda_1) for the exponential model with lambda_1
 * the lowest x1 bound state of the exact axis.  V12 is the model's two-body
 * potential.  Needs gamma = 0 (a real interior).  Synchronising.              */
mgc_status mgc_cross_section(mgc_grid g, const void* u, const void* chi,
                             double k1, double k2, double zeta[2], double* sigma);

/* The amplitude and cross section of mgc_cross_section for many momentum
 * pairs in one pass over the field (Sec. 3.3: the singly differential cross
 * section of an energy sharing is sigma along k1 = K cos a, k2 = K sin a,
 * K^2 / 2 the excess energy, a in [0, pi/2]):
 *   zeta[2a], zeta[2a+1] = Re, Im zeta(k1[a], k2[a]),  sigma[a] = sigma(k1[a], k2[a]).
 * k1, k2: host arrays of npairs momenta > 0; zeta: host array of 2 npairs
 * doubles; sigma: host array of npairs doubles, or NULL.  u, chi: FP64 level-0
 * fields.  1 <= npairs <= MGC_SWEEP_MAX, else MGC_EINVAL (also for a null
 * pointer or a momentum that is not positive).  Synchronising.                */
mgc_status mgc_cross_section_sweep(mgc_grid g, const void* u, const void* chi, int npairs,
                                   const double* k1, const double* k2, double* zeta, double* sigma);

/* Most bound states one single-ionisation call evaluates. */
#define MGC_SI_MAX 16

/* Single-ionisation amplitudes (Sec. 3.3 eq. single-ionization):
 *   s_n = sum_{j,k<=j0} t_j t_k phi_{k_n}(x1_j) phi_n(x2_k) (chi - V12 u)_{kj},
 * n = 1 .. nstates, with phi_n the n-th lowest bound state of the exact x2
 * one-body Hamiltonian -1/2 d2/dz2 + V2(z) of the model (eq. 1d_eigenstate on the
 * exterior-complex-scaled grid, bilinear normalisation, two shift-and-invert
 * refinement steps), k_n = sqrt(2 (E - Re lambda_n)) and phi_{k_n} the test
 * function of eq. testfunction in x1 (as in mgc_cross_section); t the
 * trapezoid weights of the real region.  s: host array of 2 nstates doubles
 * (Re, Im of s_n); kn: host array of nstates momenta, or NULL.  u, chi: FP64
 * level-0 fields.  MGC_EINVAL for nstates outside [1, MGC_SI_MAX] (or not
 * below n - 1) or a closed channel (E <= Re lambda_n).  One pass over the
 * field for all states.  Synchronising.                                      */
mgc_status mgc_single_ionization(mgc_grid g, const void* u, const void* chi, int nstates, double* s, double* kn);

/* Total double-ionisation cross section (Sec. 3.3 eq. total-double-ionization)
 *   sigma_tot(E) = int_0^E sigma(sqrt(2 eps), sqrt(2 (E - eps))) d eps
 * with eps = E sin^2 a (k1 = sqrt(2E) sin a, k2 = sqrt(2E) cos a), where the
 * Jacobian 2E sin a cos a cancels the 1/(k1 k2) of sigma:
 *   sigma_tot = 8 pi^2 / k0^2 int_0^{pi/2} |zeta(k1(a), k2(a))|^2 da,
 * by a nodes-point Gauss-Legendre rule in a (all amplitudes in one pass over
 * the field).  zeta: host array of 2 nodes doubles receiving the amplitudes at
 * the nodes (ascending a), or NULL.  MGC_EINVAL for nodes outside
 * [1, MGC_SWEEP_MAX] or E <= 0.  Synchronising.                              */
mgc_status mgc_total_double_ionization(mgc_grid g, const void* u, const void* chi, int nodes, double* sigma_tot,
                                       double* zeta);

/* Gradient of sigma(k1, k2) with respect to (Z1, Z2, lambda) for u = A^{-1} chi,
 * chi the Temkin-Poet right-hand side of mgc_build_rhs_tp (call order:
 * set_potential, set_energy, build_rhs_tp, solve, then this).  The complex
 * symmetry of Sec. 2.5 gives the adjoint: A^T v = d zeta/du is solved with
 * mgc_solve_transpose (opts, stats; v: initial guess in, adjoint solution out,
 * an FP64 level-0 field), then
 *   d zeta/dp = sum F' (chi - V12 u) + sum F (dchi/dp - dV12/dp u)
 *             + sum v (dchi/dp - dA/dp u)            (no complex conjugation),
 *   d sigma/dp = 2 C Re(conj(zeta) d zeta/dp) + |zeta|^2 dC/dp,
 * C = 8 pi^2 / (k0^2 k1 k2), k0^2 = 2E + Z1^2; F = weighted phi_{k2} x phi_{k1}
 * with F' from forward-mode differentiation of the test-function recurrence.
 * Needs Z1 > 0.  Returns MGC_ENOCONV if the adjoint solve did not converge
 * (dsigma is still filled).  Synchronising.                                   */
mgc_status mgc_cross_section_grad(mgc_grid g, const void* u, const void* chi, double k1, double k2,
                                  const mgc_solve_opts* opts, void* v, double dsigma[3],
                                  double zeta[2], double* sigma, mgc_stats* stats);

/* Kernel timing (measurement support; no effect on results).
 * mgc_set_kernel_timer selects one kernel class.  While it is selected, its
 * launches inside the FGMRES restart cycles of mgc_solve and
 * mgc_solve_transpose are bracketed by HIP events recorded on the stream the
 * kernels run on (event nodes inside the captured restart graphs), in every
 * fourth restart cycle of a solve (the first included; the other cycles
 * replay a graph without timer nodes, so that the nodes' own cost stays out
 * of three quarters of the run): every Arnoldi step for the classes that
 * depend on the step (APPLY_DOT, AXPY), the first step of the cycle for the
 * others.  S1 and S2 launches of
 * all levels follow each other, so one event pair brackets each such run.
 * Right before each bracket a second event pair brackets nothing: its
 * duration (floor_ms) is what the event nodes alone add to a bracket, and
 * total_ms - floor_ms is the kernels' time as the events see it (on the
 * timed 1025^2 workload a few microseconds per launch below the profiler's
 * kernel duration: the bracket's start overlaps the kernel's dispatch).
 * The durations, the launch count and the kernels' algorithmic bytes
 * (compulsory loads and stores of their operands over the interior nodes)
 * accumulate until mgc_read_kernel_timer, which returns and clears them.
 * MGC_KT_NONE turns timing off.  A new selection re-captures the restart
 * graph.  MGC_EINVAL for an unknown class, MGC_EHIP if events cannot be
 * created.                                                                    */
typedef enum {
  MGC_KT_NONE = 0,
  MGC_KT_APPLY_DOT = 1,      /* exact operator + basis dots, each Arnoldi step */
  MGC_KT_AXPY = 2,           /* first orthogonalisation axpy pass             */
  MGC_KT_S1 = 3,             /* smoothing, residual, restriction (all levels)  */
  MGC_KT_S2 = 4,             /* prolongation, post-smoothing (all levels)      */
  MGC_KT_CCCS_PROJECT = 5,   /* CCCS residual + channel projections            */
  MGC_KT_CCCS_CHAIN = 6,     /* CCCS chunk-local channel solves                */
  MGC_KT_S1_FINE = 7,        /* the finest level's S1 launch alone             */
  MGC_KT_S2_FINE = 8,        /* the finest level's S2 launch alone             */
  MGC_KT_CCCS_EXPAND = 9     /* CCCS expansion u += e* (Sec. 4.3 eq. cccs)      */
} mgc_kernel_class;
typedef struct {
  double total_ms;           /* summed event durations                         */
  long long launches;
  double bytes;              /* summed algorithmic bytes                       */
  double floor_ms;           /* summed durations of the empty event pairs      */
} mgc_kernel_timing;
mgc_status mgc_set_kernel_timer(mgc_grid g, int kernel_class);
mgc_status mgc_read_kernel_timer(mgc_grid g, mgc_kernel_timing* out);

/* Batched solves (many energies and grid sizes at once).
 * A batch groups `count` handles that live on one device, each with its own
 * workspace, potential and energy already set (the handles stay owned by the
 * caller and must outlive the batch).  mgc_batch_solve runs FGMRES (opts->outer
 * must be MGC_FGMRES) on all of them together: each unfinished solve's
 * restart cycle, its true residual and a three-number report are captured
 * into one graph per solve; each round launches these graphs over 4
 * library-owned streams (default priority) so that they run concurrently and
 * synchronises once, then reads the reports.  Finished solves drop out.  The
 * initial residuals run on the first handle's stream, which the side streams
 * wait for.  u[i] (initial guess in, solution out) and f[i] are FP64 level-0
 * fields of handle i; stats (nullable) receives one entry per solve, with
 * t_solve_ms the wall time of the whole batch.  Each solve performs the same
 * arithmetic as mgc_solve on its handle, so it reaches the same iterate.
 * Returns MGC_OK when every solve converged, otherwise the first failing
 * status in handle order (per-solve iterations and residuals are in stats
 * either way).  No device memory is allocated.                               */
typedef struct mgc_batch_s* mgc_batch;
mgc_status mgc_batch_create(const mgc_grid* grids, int count, mgc_batch* out);
mgc_status mgc_batch_solve(mgc_batch b, void* const* u, const void* const* f,
                           const mgc_solve_opts* opts, mgc_stats* stats);
/* The cross sections of every solve of a batch (the energies of a batch in
 * one call): for handle i, sigma_tot[i] as mgc_total_double_ionization with
 * `nodes` points (skipped for nodes = 0) and s[2 nstates i ..] as
 * mgc_single_ionization with `nstates` states (skipped for nstates = 0).  The
 * sweeps of the handles run concurrently on the batch's streams after the
 * work already queued on the handles' streams; one synchronisation.        */
mgc_status mgc_batch_cross_sections(mgc_batch b, const void* const* u, const void* const* chi, int nodes,
                                    int nstates, double* sigma_tot, double* s);
mgc_status mgc_batch_destroy(mgc_batch b);

mgc_status mgc_destroy_grid(mgc_grid g);

/* Thread-local description of the last error (never NULL).                  */
const char* mgc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MGCCCS_H */
