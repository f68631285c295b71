// C ABI of the MG-CCCS solver (include/mgcccs.h): handle management,
// workspace layout, setup upload and the host-side drivers of the V-cycle,
// the Coupled Channel Correction Step and the outer iterations.
#include "../../include/mgcccs.h"

#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "internal.h"
#include "launch.h"
#include "setup.h"

using namespace mgc;

namespace {

thread_local std::string g_err = "no error";

mgc_status fail(mgc_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

constexpr int P64 = 0, P32 = 1;
inline size_t esize(int prec) { return prec == P64 ? 16 : 8; }
inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct LevelInfo {
  int n = 0, pitch = 0;
  Axis ax;                                 // axis of this hierarchy level
  size_t tab[2] = {0, 0};                  // 5 tables a, c, px, py, tm (per precision)
  size_t fu[2] = {0, 0}, ff[2] = {0, 0}, ft[2] = {0, 0};  // fields
  size_t gsV[2] = {0, 0}, gsst[2] = {0, 0};               // GMRES(3) smoother: 4 fields, state
  size_t v12[2] = {0, 0};                  // general two-body table (pot_tables)
};

// Potential model of a handle: Temkin-Poet (-Z1/x1, -Z2/x2, lambda/max) or the
// exponential model (-a1 exp(-b1 x1^2), -a2 exp(-b2 x2^2),
// c12 exp(-d12 (x1 + x2)^2)), both continued onto the complex nodes.
constexpr int POT_TP = 0, POT_EXP = 1;
struct PotModel {
  int kind = POT_TP;
  double Z1 = 1, Z2 = 1, lam = 1;
  double a1 = 0, b1 = 0, a2 = 0, b2 = 0, c12 = 0, d12 = 0;
  cd v1(cd z) const { return kind == POT_EXP ? -a1 * std::exp(-b1 * z * z) : -Z1 / z; }
  cd v2(cd z) const { return kind == POT_EXP ? -a2 * std::exp(-b2 * z * z) : -Z2 / z; }
  // two-body value at nodes j (x1) and k (x2) of an axis
  cd v12(const Axis& ax, int j, int k) const {
    if (kind == POT_EXP) {
      const cd s = ax.z[j] + ax.z[k];
      return c12 * std::exp(-d12 * s * s);
    }
    return lam / ax.z[std::max(j, k)];
  }
};

struct SysOff {                            // offsets of one channel system's factors
  size_t G = 0, Vs = 0, Ws = 0, lo = 0, up = 0, Rinv = 0, Tif = 0, start = 0;
};

struct CcOff {                             // CCCS tables + scratch for one precision
  size_t wphi = 0, phi = 0, wvphi = 0, vphi = 0;
  SysOff A, B;
  size_t partA = 0, partB = 0, rhoA = 0, rhoB = 0, partC = 0, gA = 0, gB = 0,
         YA = 0, YB = 0, HA = 0, HB = 0, eA = 0, eB = 0;
};

}  // namespace

struct GraphCache {                       // one captured FGMRES restart cycle
  hipGraphExec_t exec = nullptr;
  const void* u = nullptr;
  const void* f = nullptr;
  int m = 0, mm = 0, inner = -1, kt = 0;
  double tol_abs = 0;
  int kt_slots = 0;                        // timer slots recorded in the graph
  std::vector<double> kt_bytes;
  std::vector<int> kt_count;
};

// Event timing of one kernel class (mgc_set_kernel_timer).  Slots are event
// pairs handed out in launch order during one restart cycle's enqueue; a slot
// brackets one launch or a run of consecutive launches of the class (count).
// Event record nodes cost a few microseconds each inside a graph, so classes
// whose launches do not depend on the Arnoldi step are timed in the first
// step of each restart cycle only (`open`).  Right before each bracket a
// second pair (fev) brackets one empty launch: what the event nodes and a
// launch add to a bracket, subtracted from the bracketed time.
constexpr int KT_SAMPLE = 4;               // restart cycles per timed one
struct KernelTimer {
  static constexpr int SLOTS = 4 * MGC_MAX_RESTART;
  int which = MGC_KT_NONE;
  hipEvent_t ev[2 * SLOTS] = {};
  hipEvent_t fev[2 * SLOTS] = {};
  std::vector<double> bytes = std::vector<double>(SLOTS, 0.0);
  std::vector<int> count = std::vector<int>(SLOTS, 0);
  int used = 0;
  bool open = true;                        // slots may be handed out in this step
  int run = -1;                            // slot of the S1 / S2 run in progress
  double ms = 0, floor_ms = 0, total_bytes = 0;
  long long launches = 0;
};

struct mgc_grid_s {
  mgc_grid_desc d{};
  mgc_schedule sched{-1, 1, 1};            // launch schedule (mgc_set_schedule)
  hipStream_t stream = nullptr;
  hipStream_t cap = nullptr;               // capture stream (default priority)
  GraphCache graph;                        // restart cycle (with the timer's nodes when one is selected)
  GraphCache plain;                        // the same cycle without timer nodes (unsampled cycles)
  GraphCache bicg_graph;                   // one captured BiCGSTAB iteration
  KernelTimer kt;
  int device = 0;
  bool failed = false;
  Axis exact;                              // level-0 axis of the physical operator
  std::vector<LevelInfo> lv;
  int PA = 1, PB = 1;                      // channel chunks of the A / B systems
  // setup state
  bool have_pot = false, have_energy = false;
  double Z1 = 1, Z2 = 1, lam = 1, E = 0;
  PotModel pot;                            // the model set by mgc_set_potential / mgc_set_potential_exp
  std::vector<cd> lamA, lamB;
  std::vector<std::vector<cd>> phi, vphi;
  double t_setup_ms = 0;
  // workspace
  char* ws = nullptr;
  size_t ws_bytes = 0, need = 0;
  size_t exact_tab = 0, exact_tab32 = 0, exact_w = 0, exact_z = 0, coarse_inv = 0, tt = 0;
  size_t exact_v12[2] = {0, 0};            // two-body table of the physical operator (pot_tables)
  CcOff cc[2];
  size_t part = 0, scal = 0;               // reduction partials, small scalars
  size_t gspart = 0;                       // partials of the GMRES(3) smoother
  size_t dfl[2] = {0, 0};                  // deflation-ordered preconditioner: residual, V-cycle correction
  size_t apart = 0;                        // 3 x ARNOLDI_PART partials of the Arnoldi passes
  bool basis_dirty = false;                // Krylov basis may hold non-finite values
  size_t r64 = 0, f32 = 0, u32 = 0, tw = 0, tz = 0;
  size_t W = 0, Z[2] = {0, 0};
  size_t gm = 0;                           // GmresState arrays
  size_t zeta_f = 0, adj = 0;
  size_t sweep_f = 0, sweep_k = 0, sweep_part = 0, sweep_out = 0;   // mgc_cross_section_sweep
  size_t si_tab = 0;                       // bound states of the exact x2 Hamiltonian (single ionisation)
  size_t v1r = 0, tm0 = 0;                 // V1 at the real nodes of the exact axis; a zero two-body table
  std::vector<double> v1r_host;
  double lam1x = 0;                        // lowest x1 bound state of the exact axis (exponential model)
  int si_count = 0;                        // states held in si_tab (0: none for this potential)
  std::vector<cd> si_lam;
  int nchunksB = 1;
  bool prec_on[2] = {true, false};

  int coarsest() const { return (int)lv.size() - 1; }
  size_t field_bytes(int l, int prec) const { return (size_t)(lv[l].n + 1) * lv[l].pitch * esize(prec); }
  template <typename T> T* at(size_t off) const { return reinterpret_cast<T*>(ws + off); }
};

namespace {

bool hip_ok(mgc_grid g, hipError_t e, const char* what) {
  if (e == hipSuccess) return true;
  g->failed = true;
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  return false;
}
#define HIPCHK(g, call)                                  \
  do {                                                   \
    if (!hip_ok((g), (call), #call)) return MGC_EHIP;    \
  } while (0)

// A captured restart cycle bakes E and the table pointers into its kernel
// arguments: any setup change invalidates it.
void drop_graph(mgc_grid g) {
  if (g->graph.exec) (void)hipGraphExecDestroy(g->graph.exec);
  g->graph = GraphCache();
  if (g->plain.exec) (void)hipGraphExecDestroy(g->plain.exec);
  g->plain = GraphCache();
  if (g->bicg_graph.exec) (void)hipGraphExecDestroy(g->bicg_graph.exec);
  g->bicg_graph = GraphCache();
}

inline int pitch_for(int n) { return ((n + 1) + 15) / 16 * 16; }

// --------------------------------------------------------------------------
// workspace layout
// The scratch of one CCCS application (partials, channel vectors) for
// precision p, placed by take(bytes) -> offset.
template <typename Take> void cccs_scratch_layout(const mgc_grid_s* g, int p, Take& take, CcOff& c) {
  const int n = g->d.n, N = n - 1, M = g->d.M, Lc = g->d.Lch;
  const size_t e = esize(p);
  c.partA = take((size_t)g->nchunksB * (n + 1) * M * e);
  c.partB = take((size_t)g->nchunksB * (n + 1) * Lc * e);
  c.rhoA = take((size_t)(n + 1) * M * e);
  c.rhoB = take((size_t)(n + 1) * Lc * e);
  c.partC = take((size_t)launch_cccs_reduce_blocks(n) * M * Lc * e);
  c.gA = take((size_t)N * M * e);
  c.gB = take((size_t)N * Lc * e);
  c.YA = take((size_t)g->PA * 2 * M * e);
  c.YB = take((size_t)g->PB * 2 * Lc * e);
  c.HA = take((size_t)g->PA * 4 * M * e);
  c.HB = take((size_t)g->PB * 4 * Lc * e);
  c.eA = take((size_t)(n + 1) * M * e);
  c.eB = take((size_t)(n + 1) * Lc * e);
}

void layout(mgc_grid g) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  const int n = g->d.n, N = n - 1, M = g->d.M, Lc = g->d.Lch;
  g->exact_tab = take(5 * (n + 1) * 16);
  if (g->prec_on[P32]) g->exact_tab32 = take(5 * (n + 1) * 8);
  g->exact_w = take((n + 1) * 16);
  g->exact_z = take((n + 1) * 16);
  for (int p = 0; p < 2; ++p) {
    if (!g->prec_on[p]) continue;
    if (g->d.pot_tables) g->exact_v12[p] = take(g->field_bytes(0, p));
    for (size_t l = 0; l < g->lv.size(); ++l) {
      LevelInfo& L = g->lv[l];
      L.tab[p] = take(5 * (L.n + 1) * esize(p));
      if (g->d.pot_tables) L.v12[p] = take(g->field_bytes((int)l, p));
      const size_t fb = g->field_bytes((int)l, p);
      if (l > 0) { L.fu[p] = take(fb); L.ff[p] = take(fb); }
      L.ft[p] = take(fb);
      if (g->d.smoother == MGC_SMOOTH_GMRES3 && (int)l >= g->d.gs_from && (int)l + 1 < (int)g->lv.size()) {
        L.gsV[p] = take(4 * fb);
        L.gsst[p] = take(32 * sizeof(double));
      }
    }
    CcOff& c = g->cc[p];
    const size_t e = esize(p);
    if (M > 0 || Lc > 0) {
      c.wphi = take((size_t)M * (n + 1) * e);
      c.phi = take((size_t)M * (n + 1) * e);
      c.wvphi = take((size_t)Lc * (n + 1) * e);
      c.vphi = take((size_t)Lc * (n + 1) * e);
      auto sys = [&](SysOff& s, int m, int P) {
        s.G = take((size_t)N * m * m * e);
        s.Vs = take((size_t)N * m * m * e);
        s.Ws = take((size_t)N * m * m * e);
        s.lo = take((size_t)N * e);
        s.up = take((size_t)N * e);
        const size_t RR = (size_t)4 * m * m;
        s.Rinv = take((size_t)(P > 1 ? P - 1 : 1) * RR * e);
        const size_t QR = (size_t)(P > 1 ? P - 1 : 1) * 2 * m;
        s.Tif = take(QR * QR * e);
        s.start = take((size_t)(P + 1) * sizeof(int));
      };
      sys(c.A, M, g->PA);
      sys(c.B, Lc, g->PB);
      cccs_scratch_layout(g, p, take, c);
    }
  }
  const int nc = g->lv.back().n, Nc = (nc - 1) * (nc - 1);
  g->coarse_inv = take((size_t)Nc * Nc * 16);
  const int nb = std::max(launch_stencil_blocks(n), launch_vec_blocks(n));
  g->part = take((size_t)nb * 64 * sizeof(double));
  if (g->d.smoother == MGC_SMOOTH_GMRES3) g->gspart = take((size_t)gmres3_part_doubles(n) * sizeof(double));
  if (g->d.pc_order == MGC_PC_DEFLATION)
    for (int p = 0; p < 2; ++p)
      if (g->prec_on[p]) g->dfl[p] = take(2 * g->field_bytes(0, p));
  g->scal = take(256 * sizeof(double));
  g->apart = take((size_t)3 * ARNOLDI_PART * sizeof(double));
  g->r64 = take(g->field_bytes(0, P64));
  g->tw = take(g->field_bytes(0, P64));
  g->tz = take(g->field_bytes(0, P64));
  g->tt = take(g->field_bytes(0, P64));
  if (g->prec_on[P32]) {
    g->f32 = take(g->field_bytes(0, P32));
    g->u32 = take(g->field_bytes(0, P32));
  }
  const int m = g->d.max_restart;
  if (m > 0) {
    g->W = take((size_t)(m + 1) * g->field_bytes(0, P64));
    for (int p = 0; p < 2; ++p)
      if (g->prec_on[p]) g->Z[p] = take((size_t)m * g->field_bytes(0, p));
  }
  g->gm = take((size_t)(16 * (m + 2) + 2 * (m + 1) * (m + 1) + 64) * sizeof(double));
  g->zeta_f = take(4 * (n + 1) * sizeof(double));
  g->adj = take(g->field_bytes(0, P64));
  g->sweep_f = take((size_t)2 * (n + 1) * MGC_SWEEP_MAX * sizeof(double));
  g->sweep_part = take((size_t)zeta_sweep_blocks(n) * 2 * MGC_SWEEP_MAX * sizeof(double));
  g->sweep_out = take((size_t)2 * MGC_SWEEP_MAX * sizeof(double));
  g->sweep_k = take((size_t)2 * MGC_SWEEP_MAX * sizeof(double));
  g->si_tab = take((size_t)MGC_SI_MAX * (n + 1) * 16);
  g->v1r = take((size_t)(n + 1) * sizeof(double));
  g->tm0 = take((size_t)(n + 1) * 16);
  g->need = off;
}

GmresState gmres_state(mgc_grid g) {
  const int m = std::max(g->d.max_restart, 1);
  double* b = g->at<double>(g->gm);
  GmresState s;
  size_t o = 0;
  auto take = [&](size_t cnt) { double* p = b + o; o += cnt; return p; };
  s.hcol = take(2 * (m + 1));
  s.nrm2 = take(2);
  s.scale = take(m + 2);
  s.H = take(2 * (m + 1) * m);
  s.cs = take(2 * m);
  s.sn = take(2 * m);
  s.g = take(2 * (m + 1));
  s.est = take(m);
  s.y = take(2 * m);
  s.upcoef = reinterpret_cast<double2*>(take(2 * m));
  s.beta = take(2);
  s.kstar = reinterpret_cast<int*>(take(2));
  s.kused = reinterpret_cast<int*>(take(2));
  s.ticket = reinterpret_cast<unsigned*>(take(2));
  return s;
}

template <typename T> Level<T> level_of(mgc_grid g, int l) {
  const int p = sizeof(T) == 8 ? P64 : P32;
  const LevelInfo& L = g->lv[l];
  const size_t e = esize(p), sz = (size_t)(L.n + 1) * e;
  Level<T> out;
  const char* base = g->ws + L.tab[p];
  out.a = (const v2<T>*)(base);
  out.c = (const v2<T>*)(base + sz);
  out.px = (const v2<T>*)(base + 2 * sz);
  out.py = (const v2<T>*)(base + 3 * sz);
  out.tm = (const v2<T>*)(base + 4 * sz);
  out.v12 = g->pot.kind == POT_EXP ? (const v2<T>*)(g->ws + L.v12[p]) : nullptr;
  out.n = L.n;
  out.pitch = L.pitch;
  out.E = (T)g->E;
  return out;
}

template <typename T = double> Level<T> exact_level(mgc_grid g) {
  const int n = g->d.n;
  const size_t sz = (size_t)(n + 1) * sizeof(v2<T>);
  const char* base = g->ws + (sizeof(T) == 8 ? g->exact_tab : g->exact_tab32);
  Level<T> out;
  out.a = (const v2<T>*)(base);
  out.c = (const v2<T>*)(base + sz);
  out.px = (const v2<T>*)(base + 2 * sz);
  out.py = (const v2<T>*)(base + 3 * sz);
  out.tm = (const v2<T>*)(base + 4 * sz);
  out.v12 = g->pot.kind == POT_EXP ? (const v2<T>*)(g->ws + g->exact_v12[sizeof(T) == 8 ? P64 : P32]) : nullptr;
  out.n = n;
  out.pitch = g->lv[0].pitch;
  out.E = (T)g->E;
  return out;
}

template <typename T> ChanTab<T> chan_of(mgc_grid g) {
  const int p = sizeof(T) == 8 ? P64 : P32;
  const CcOff& c = g->cc[p];
  ChanTab<T> t;
  t.wphi = g->at<const v2<T>>(c.wphi);
  t.phi = g->at<const v2<T>>(c.phi);
  t.wvphi = g->at<const v2<T>>(c.wvphi);
  t.vphi = g->at<const v2<T>>(c.vphi);
  t.M = g->d.M;
  t.L = g->d.Lch;
  return t;
}

template <typename T> ChanSys<T> sys_of(mgc_grid g, bool A) {
  const int p = sizeof(T) == 8 ? P64 : P32;
  const SysOff& s = A ? g->cc[p].A : g->cc[p].B;
  ChanSys<T> o;
  o.G = g->at<const v2<T>>(s.G);
  o.Vs = g->at<const v2<T>>(s.Vs);
  o.Ws = g->at<const v2<T>>(s.Ws);
  o.lo = g->at<const v2<T>>(s.lo);
  o.up = g->at<const v2<T>>(s.up);
  o.Rinv = g->at<const v2<T>>(s.Rinv);
  o.Tif = g->at<const v2<T>>(s.Tif);
  o.start = g->at<const int>(s.start);
  o.N = g->d.n - 1;
  o.M = A ? g->d.M : g->d.Lch;
  o.P = A ? g->PA : g->PB;
  return o;
}

CccsScratch scratch_at(char* base, const CcOff& c) {
  CccsScratch w;
  w.partA = base + c.partA;
  w.partB = base + c.partB;
  w.rhoA = base + c.rhoA;
  w.rhoB = base + c.rhoB;
  w.partC = base + c.partC;
  w.gA = base + c.gA;
  w.gB = base + c.gB;
  w.YA = base + c.YA;
  w.YB = base + c.YB;
  w.HA = base + c.HA;
  w.HB = base + c.HB;
  w.eA = base + c.eA;
  w.eB = base + c.eB;
  return w;
}
CccsScratch scratch_of(mgc_grid g, int p) { return scratch_at(g->ws, g->cc[p]); }

// --------------------------------------------------------------------------
// uploads
template <typename T> std::vector<v2<T>> cast_vec(const std::vector<cd>& v) {
  std::vector<v2<T>> o(v.size());
  for (size_t i = 0; i < v.size(); ++i) { o[i].x = (T)v[i].real(); o[i].y = (T)v[i].imag(); }
  return o;
}

mgc_status upload(mgc_grid g, size_t off, const void* src, size_t bytes) {
  HIPCHK(g, hipMemcpyAsync(g->ws + off, src, bytes, hipMemcpyHostToDevice, g->stream));
  HIPCHK(g, hipStreamSynchronize(g->stream));   // host vectors are temporaries
  return MGC_OK;
}

template <typename T> mgc_status upload_cplx(mgc_grid g, size_t off, const std::vector<cd>& v) {
  auto c = cast_vec<T>(v);
  return upload(g, off, c.data(), c.size() * sizeof(v2<T>));
}

std::vector<cd> one_body(const Axis& ax, double Z) {
  std::vector<cd> V(ax.n + 1, 0.0);
  for (int j = 1; j < ax.n; ++j) V[j] = -Z / ax.z[j];
  return V;
}
// V1 (coord 1) or V2 (coord 2) of the model on the interior nodes of an axis
std::vector<cd> one_body(const Axis& ax, const PotModel& m, int coord) {
  std::vector<cd> V(ax.n + 1, 0.0);
  for (int j = 1; j < ax.n; ++j) V[j] = coord == 1 ? m.v1(ax.z[j]) : m.v2(ax.z[j]);
  return V;
}

// a, c, px, py, tm for an axis (concatenated); tm is zero for a model whose
// two-body part lives in the general table
std::vector<cd> level_tables(const Axis& ax, const PotModel& m) {
  const int n = ax.n;
  std::vector<cd> t(5 * (n + 1), 0.0);
  for (int j = 1; j < n; ++j) {
    t[j] = ax.a[j];
    t[(n + 1) + j] = ax.c[j];
    t[2 * (n + 1) + j] = ax.b[j] + m.v1(ax.z[j]);
    t[3 * (n + 1) + j] = ax.b[j] + m.v2(ax.z[j]);
    t[4 * (n + 1) + j] = m.kind == POT_TP ? m.lam / ax.z[j] : cd(0.0);
  }
  return t;
}
// general two-body table V12(z_j, z_k) at [k][j] (pitch columns), zero on the ring
std::vector<cd> two_body_table(const Axis& ax, const PotModel& m, int pitch) {
  const int n = ax.n;
  std::vector<cd> t((size_t)(n + 1) * pitch, 0.0);
  for (int k = 1; k < n; ++k)
    for (int j = 1; j < n; ++j) t[(size_t)k * pitch + j] = m.v12(ax, j, k);
  return t;
}

mgc_status check_ready(mgc_grid g, bool need_energy = true) {
  if (!g) return fail(MGC_EINVAL, "null handle");
  if (g->failed) return fail(MGC_ESTATE, "handle failed after an earlier HIP error: " + g_err);
  if (!g->ws) return fail(MGC_ESTATE, "no workspace bound");
  if (need_energy && !g->have_energy) return fail(MGC_ESTATE, "set_potential and set_energy required");
  return MGC_OK;
}

// --------------------------------------------------------------------------
// V-cycle and CCCS drivers
// Kernel timer hooks.  kt_slot hands out the next event pair for a launch of
// class `kind` (-1: that class is not being timed); kt_mark records one end.
int kt_slot(mgc_grid g, int kind, double bytes) {
  KernelTimer& t = g->kt;
  if (t.which == MGC_KT_NONE || t.which != kind || !t.open || t.used >= KernelTimer::SLOTS) return -1;
  t.bytes[t.used] = bytes;
  t.count[t.used] = 1;
  return t.used++;
}
// While the stream is being captured the event becomes an explicit event
// record node appended to the capture's current dependencies.
void kt_record(mgc_grid g, hipStream_t s, hipEvent_t ev);
void kt_mark(mgc_grid g, hipStream_t s, int slot, int end) {
  if (slot < 0) return;
  if (!end) {                              // an event pair around nothing: the pair's own cost
    kt_record(g, s, g->kt.fev[2 * slot]);
    kt_record(g, s, g->kt.fev[2 * slot + 1]);
  }
  kt_record(g, s, g->kt.ev[2 * slot + end]);
}
void kt_record(mgc_grid g, hipStream_t s, hipEvent_t ev) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (!hip_ok(g, hipStreamIsCapturing(s, &cs), "timer: capture state")) return;
  if (cs != hipStreamCaptureStatusActive) {
    (void)hip_ok(g, hipEventRecord(ev, s), "timer: event record");
    return;
  }
  hipGraph_t graph = nullptr;
  const hipGraphNode_t* deps = nullptr;
  size_t nd = 0;
  if (!hip_ok(g, hipStreamGetCaptureInfo_v2(s, &cs, nullptr, &graph, &deps, &nd), "timer: capture info")) return;
  hipGraphNode_t node;
  if (!hip_ok(g, hipGraphAddEventRecordNode(&node, graph, deps, nd, ev), "timer: event node")) return;
  (void)hip_ok(g, hipStreamUpdateCaptureDependencies(s, &node, 1, hipStreamSetCaptureDependencies),
               "timer: capture dependencies");
}
// After the stream has synchronised: add up the first `slots` event pairs.
void kt_harvest(mgc_grid g, int slots, const std::vector<double>& bytes, const std::vector<int>& count) {
  KernelTimer& t = g->kt;
  for (int i = 0; i < slots; ++i) {
    float ms = 0.0f, fl = 0.0f;
    if (hipEventElapsedTime(&ms, t.ev[2 * i], t.ev[2 * i + 1]) != hipSuccess) continue;
    if (hipEventElapsedTime(&fl, t.fev[2 * i], t.fev[2 * i + 1]) != hipSuccess) continue;
    t.ms += ms;
    t.floor_ms += fl;
    t.total_bytes += bytes[i];
    t.launches += count[i];
  }
}

// Fused zero-guess cycle: does level l take the small tiles (fewer than two
// large tiles per CU), is it in the coarse tail, and is it the finer level of
// a pair whose S2 passes share one launch (pairs counted from the first
// small-tile level, both members above the tail)?
// The schedule (mgc_set_schedule) decides the tile size per level, and
// whether pairs and the tail are used; every choice gives the same results
// bit for bit (the tests compare them).
// GMRES(3) smoothing on level l (the levels from gs_from on, with the GMRES(3)
// smoother selected); any_gs: some level above the coarsest takes it
bool gs_level(mgc_grid g, int l) { return g->d.smoother == MGC_SMOOTH_GMRES3 && l >= g->d.gs_from; }
bool any_gs(mgc_grid g) { return gs_level(g, g->coarsest() - 1); }
bool small_tiles(mgc_grid g, int l) {
  if (g->sched.small_tiles >= 0) return l < 31 && ((g->sched.small_tiles >> l) & 1);
  const int n = g->lv[l].n;
  return (long long)((n - 1 + 63) / 64) * ((n - 1 + 15) / 16) < 512;
}
bool in_tail(mgc_grid g, int l) {
  return g->sched.coarse_tail && !any_gs(g) && g->lv[l].n <= TAIL_MAX_N && g->coarsest() - l <= TMAXL;
}
bool pair_level(mgc_grid g, int l) {
  if (!g->sched.level_pairs) return false;
  if (l + 1 >= g->coarsest() || in_tail(g, l) || in_tail(g, l + 1) || !small_tiles(g, l) || gs_level(g, l + 1))
    return false;
  int s0 = l;
  while (s0 > 0 && small_tiles(g, s0 - 1)) --s0;
  return (l - s0) % 2 == 0;
}

template <typename T>
void vcycle_level(mgc_grid g, int l, void* u, const void* f, bool zero_guess, const double* fs = nullptr) {
  const int p = sizeof(T) == 8 ? P64 : P32;
  hipStream_t s = g->stream;
  Level<T> L = level_of<T>(g, l);
  if (l == g->coarsest()) {
    launch_coarse_solve<T>(s, g->at<const double2>(g->coarse_inv), L.n, L.pitch, f, u);
    return;
  }
  const LevelInfo& LI = g->lv[l];
  const LevelInfo& LC = g->lv[l + 1];
  const double om = g->d.omega;
  if (gs_level(g, l) && g->sched.coarse_tail && LI.n <= GT_MAX_N && g->coarsest() - l <= TMAXL) {
    // this level and every coarser one in one single-workgroup launch
    GsTailArgs<T> A{};
    const int nl = g->coarsest() - l;
    for (int i = 0; i < nl; ++i) A.L[i] = level_of<T>(g, l + i);
    A.f0 = static_cast<const v2<T>*>(f);
    A.u0 = static_cast<v2<T>*>(u);
    for (int i = 1; i <= nl; ++i) {
      A.f[i] = g->at<v2<T>>(g->lv[l + i].ff[p]);
      A.u[i] = g->at<v2<T>>(g->lv[l + i].fu[p]);
      A.pitch[i] = g->lv[l + i].pitch;
    }
    A.nl = nl;
    A.nc = g->lv[g->coarsest()].n;
    A.Ainv = g->at<const double2>(g->coarse_inv);
    A.zero = zero_guess ? 1 : 0;
    A.nu1 = g->d.nu1;
    A.nu2 = g->d.nu2;
    launch_gs_tail<T>(s, A);
    return;
  }
  if (gs_level(g, l)) {
    // GMRES(3) smoothing substitute: in place on u, per level
    void* V = g->ws + LI.gsV[p];
    const size_t stride = g->field_bytes(l, p) / sizeof(v2<T>);
    double* st = g->at<double>(LI.gsst[p]);
    double* part = g->at<double>(g->gspart);
    if (zero_guess) launch_fill_zero(s, u, g->field_bytes(l, p));
    for (int it = 0; it < g->d.nu1; ++it) launch_gmres3_smooth<T>(s, L, u, f, V, stride, st, part);
    launch_resid_restrict<T>(s, L, u, f, g->ws + LC.ff[p], LC.pitch);
    vcycle_level<T>(g, l + 1, g->ws + LC.fu[p], g->ws + LC.ff[p], true);
    launch_prolong_add<T>(s, L.n, L.pitch, u, g->ws + LC.fu[p], LC.pitch);
    for (int it = 0; it < g->d.nu2; ++it) launch_gmres3_smooth<T>(s, L, u, f, V, stride, st, part);
    return;
  }
  if (zero_guess && g->d.nu1 == 1 && g->d.nu2 == 1) {
    // fused passes: u' = omega f/d is recomputed, never stored
    const double Nf = (double)(L.n - 1) * (L.n - 1), Nc = (double)(L.n / 2 - 1) * (L.n / 2 - 1);
    const double e = (double)sizeof(v2<T>);
    // timing: the S1 launches of all levels run back to back (one event
    // pair around them), and so do the S2 launches
    KernelTimer& kt = g->kt;
    if (l == 0) {
      kt.run = kt_slot(g, MGC_KT_S1, 0.0);
      if (kt.run >= 0) kt.count[kt.run] = 0;
      kt_mark(g, s, kt.run, 0);
    }
    const int nl = g->coarsest() - l;
    if (L.n <= TAIL_MAX_N && nl <= TMAXL && g->sched.coarse_tail && !any_gs(g)) {
      // coarse tail: every remaining level in two launches
      TailArgs<T> A{};
      double b1 = 0.0, b2 = 0.0;
      for (int i = 0; i <= nl; ++i) {
        const LevelInfo& Li = g->lv[l + i];
        if (i < nl) {
          A.L[i] = level_of<T>(g, l + i);
          const double nf = (double)(Li.n - 1) * (Li.n - 1), nc = (double)(Li.n / 2 - 1) * (Li.n / 2 - 1);
          b1 += (nf + nc) * e;                                       // f in, f_c out
          b2 += (2 * nf + nc) * e;                                   // f, e_c in, u out
        }
        A.f[i] = (v2<T>*)(i == 0 ? (void*)f : (void*)(g->ws + Li.ff[p]));
        A.u[i] = (v2<T>*)(i == 0 ? u : (void*)(g->ws + Li.fu[p]));
        A.pitch[i] = Li.pitch;
      }
      const int ncs = g->lv[g->coarsest()].n;
      const double Ncs = (double)(ncs - 1) * (ncs - 1);
      b1 += Ncs * Ncs * 16.0 + Ncs * e;                              // Ainv in, u_c out
      A.nl = nl;
      A.nc = ncs;
      A.Ainv = g->at<const double2>(g->coarse_inv);
      A.fs = fs;
      A.omega = (T)om;
      if (kt.run >= 0 && kt.which == MGC_KT_S1) {
        kt.bytes[kt.run] += b1;
        ++kt.count[kt.run];
      }
      launch_tail<T>(s, A, true);
      if (kt.which == MGC_KT_S1) {
        kt_mark(g, s, kt.run, 1);
        kt.run = -1;
      }
      kt.run = kt_slot(g, MGC_KT_S2, 0.0);
      if (kt.run >= 0) kt.count[kt.run] = 0;
      kt_mark(g, s, kt.run, 0);
      if (kt.run >= 0 && kt.which == MGC_KT_S2) {
        kt.bytes[kt.run] += b2;
        ++kt.count[kt.run];
      }
      launch_tail<T>(s, A, false);
      if (l == 0 && kt.which == MGC_KT_S2) {
        kt_mark(g, s, kt.run, 1);
        kt.run = -1;
      }
      return;
    }
    // levels l and l+1 in one S1 and one S2 launch (small tiles, both above
    // the tail)
    const bool pair = pair_level(g, l);
    const int lnext = pair ? l + 2 : l + 1;
    const LevelInfo& LN = g->lv[lnext];
    const double N2 = (double)(LC.n / 2 - 1) * (LC.n / 2 - 1);
    if (kt.run >= 0 && kt.which == MGC_KT_S1) {
      kt.bytes[kt.run] += (Nf + Nc) * e + (pair ? N2 * e : 0.0);    // f in, f_c (and f_cc) out
      ++kt.count[kt.run];
    }
    // the finest level's launch alone (S1_FINE / S2_FINE classes)
    const int tf1 = l == 0 ? kt_slot(g, MGC_KT_S1_FINE, (Nf + Nc) * e + (pair ? N2 * e : 0.0)) : -1;
    kt_mark(g, s, tf1, 0);
    if (pair)
      launch_s1_pair<T>(s, L, level_of<T>(g, l + 1), f, fs, om, g->ws + LC.ff[p], LC.pitch, g->ws + LN.ff[p],
                        LN.pitch);
    else
      launch_s1_zero<T>(s, L, f, fs, om, g->ws + LC.ff[p], LC.pitch, small_tiles(g, l));
    kt_mark(g, s, tf1, 1);
    const bool last = lnext == g->coarsest();
    if (last && kt.which == MGC_KT_S1) {
      kt_mark(g, s, kt.run, 1);
      kt.run = -1;
    }
    vcycle_level<T>(g, lnext, g->ws + LN.fu[p], g->ws + LN.ff[p], true);
    if (last) {
      kt.run = kt_slot(g, MGC_KT_S2, 0.0);
      if (kt.run >= 0) kt.count[kt.run] = 0;
      kt_mark(g, s, kt.run, 0);
    }
    if (kt.run >= 0 && kt.which == MGC_KT_S2) {
      kt.bytes[kt.run] += (2 * Nf + Nc) * e + (pair ? N2 * e : 0.0);  // f, e_c (or f_c, e_cc) in, u out
      ++kt.count[kt.run];
    }
    const int tf2 = l == 0 ? kt_slot(g, MGC_KT_S2_FINE, (2 * Nf + Nc) * e + (pair ? N2 * e : 0.0)) : -1;
    kt_mark(g, s, tf2, 0);
    if (pair)
      launch_s2_pair<T>(s, L, level_of<T>(g, l + 1), f, fs, om, g->ws + LC.ff[p], g->ws + LN.fu[p], LN.pitch,
                        u);
    else
      launch_s2_zero<T>(s, L, f, fs, om, g->ws + LC.fu[p], LC.pitch, u, small_tiles(g, l));
    kt_mark(g, s, tf2, 1);
    if (l == 0 && kt.which == MGC_KT_S2) {
      kt_mark(g, s, kt.run, 1);
      kt.run = -1;
    }
    return;
  }
  void* bufs[2] = {u, g->ws + LI.ft[p]};
  int cur = 0;
  bool zero = zero_guess;
  for (int it = 0; it < g->d.nu1; ++it) {
    launch_jacobi<T>(s, L, zero ? nullptr : bufs[cur], f, bufs[1 - cur], om);
    zero = false;
    cur = 1 - cur;
  }
  if (zero) launch_fill_zero(s, bufs[cur], g->field_bytes(l, p));  // nu1 == 0 with a zero guess
  launch_resid_restrict<T>(s, L, bufs[cur], f, g->ws + LC.ff[p], LC.pitch);
  vcycle_level<T>(g, l + 1, g->ws + LC.fu[p], g->ws + LC.ff[p], true);
  launch_prolong_add<T>(s, L.n, L.pitch, bufs[cur], g->ws + LC.fu[p], LC.pitch);
  for (int it = 0; it < g->d.nu2; ++it) {
    launch_jacobi<T>(s, L, bufs[cur], f, bufs[1 - cur], om);
    cur = 1 - cur;
  }
  if (cur != 0) launch_scale_copy<T, T>(s, L.n, L.pitch, L.pitch, bufs[cur], nullptr, u);
}

template <typename T>
void cccs_apply(mgc_grid g, void* u, const void* f, const double* fs = nullptr, const CccsScratch* ext = nullptr) {
  if (g->d.M == 0 && g->d.Lch == 0) return;
  const int p = sizeof(T) == 8 ? P64 : P32;
  // timed kernel: projection (reads u, f; writes rho^A, rho^B) or chunk chains
  // (per system of Mc channels: G_t read in both sweeps, rho read, g written
  // and re-read in each sweep)
  const int n = g->d.n, M = g->d.M, Lc = g->d.Lch;
  const double e = (double)sizeof(v2<T>), N1 = n - 1;
  int kind = 0, slot = -1;
  if (g->kt.which == MGC_KT_CCCS_PROJECT) {
    kind = 1;
    slot = kt_slot(g, MGC_KT_CCCS_PROJECT, (2 * N1 * N1 + N1 * (M + Lc)) * e);
  } else if (g->kt.which == MGC_KT_CCCS_CHAIN) {
    kind = 2;
    slot = kt_slot(g, MGC_KT_CCCS_CHAIN, ((2.0 * M * M + 4.0 * M) + (2.0 * Lc * Lc + 4.0 * Lc)) * N1 * e);
  } else if (g->kt.which == MGC_KT_CCCS_EXPAND) {
    kind = 3;                              // u in and out, e^A, e^B in
    slot = kt_slot(g, MGC_KT_CCCS_EXPAND, (2 * N1 * N1 + N1 * (M + Lc)) * e);
  }
  struct Ctx { mgc_grid g; int slot; } ctx{g, slot};
  MarkHook hook;
  hook.fn = [](void* c, hipStream_t s, int end) {
    const Ctx* x = static_cast<const Ctx*>(c);
    kt_mark(x->g, s, x->slot, end);
  };
  hook.ctx = &ctx;
  hook.kind = slot >= 0 ? kind : 0;
  launch_cccs<T>(g->stream, level_of<T>(g, 0), u, f, fs, chan_of<T>(g), sys_of<T>(g, true),
                 sys_of<T>(g, false), ext ? *ext : scratch_of(g, p), &hook);
}

// One MG-CCCS cycle.  fs (nullable device scalar) scales f; the fused
// zero-guess path applies it on the fly, otherwise f is scaled into scratch.
template <typename T>
void mgcccs_cycle(mgc_grid g, void* u, const void* f, bool zero_guess, const double* fs = nullptr) {
  if (fs && !(zero_guess && g->d.nu1 == 1 && g->d.nu2 == 1 && !gs_level(g, 0))) {
    const int p = sizeof(T) == 8 ? P64 : P32;
    void* tmp = p == P64 ? (void*)(g->ws + g->tw) : (void*)(g->ws + g->f32);
    launch_scale_copy<T, T>(g->stream, g->d.n, g->lv[0].pitch, g->lv[0].pitch, f, fs, tmp);
    f = tmp;
    fs = nullptr;
  }
  vcycle_level<T>(g, 0, u, f, zero_guess, fs);
  cccs_apply<T>(g, u, f, fs);
}

// The Krylov preconditioner z = B v from zero: the MG-CCCS cycle, or with
// pc_order = MGC_PC_DEFLATION the channel correction first and one V-cycle
// from zero on the deflated residual, z = e*(v) + V(v - A e*(v)).
template <typename T>
void precondition(mgc_grid g, void* z, const void* v, const double* fs = nullptr) {
  if (g->d.pc_order != MGC_PC_DEFLATION || (g->d.M == 0 && g->d.Lch == 0)) {
    mgcccs_cycle<T>(g, z, v, true, fs);
    return;
  }
  const int p = sizeof(T) == 8 ? P64 : P32;
  const int n = g->d.n, pitch = g->lv[0].pitch;
  hipStream_t s = g->stream;
  if (fs) {
    void* tmp = p == P64 ? (void*)(g->ws + g->tw) : (void*)(g->ws + g->f32);
    launch_scale_copy<T, T>(s, n, pitch, pitch, v, fs, tmp);
    v = tmp;
  }
  launch_fill_zero(s, z, g->field_bytes(0, p));
  cccs_apply<T>(g, z, v);                                     // z1 = e*(v)
  // own buffers: the level-0 smoothing passes ping-pong through lv[0].ft
  void* r1 = g->ws + g->dfl[p];
  void* e = g->ws + g->dfl[p] + g->field_bytes(0, p);
  launch_stencil<T, T, T, T>(s, level_of<T>(g, 0), z, v, r1, 0, nullptr);   // v - A z1
  vcycle_level<T>(g, 0, e, r1, true);
  launch_add<T>(s, n, pitch, e, z);
}

// relres of (u, f) with the exact operator; r written to r64.  Synchronises.
mgc_status exact_residual(mgc_grid g, const void* u, const void* f, void* r, double* rr2, double* ff2,
                          double* copy_to = nullptr) {
  double* part = g->at<double>(g->part);
  double* out = g->at<double>(g->scal);
  Finish fin;
  fin.out = out;
  fin.copy_to = copy_to;
  launch_stencil<double, double, double, double>(g->stream, exact_level(g), u, f, r, 0, part, fin);
  double h[2];
  HIPCHK(g, hipMemcpyAsync(h, out, sizeof(h), hipMemcpyDeviceToHost, g->stream));
  HIPCHK(g, hipStreamSynchronize(g->stream));
  *rr2 = h[0];
  *ff2 = h[1];
  return MGC_OK;
}

void record(mgc_stats* st, int idx, double v) {
  if (!st) return;
  if (st->hist && idx < st->hist_cap) {
    st->hist[idx] = v;
    st->hist_len = idx + 1;
  }
}

mgc_status finish_status(double relres, double tol) {
  if (!std::isfinite(relres)) return fail(MGC_ENUMERIC, "non-finite residual");
  if (relres > tol) return fail(MGC_ENOCONV, "iteration limit reached");
  return MGC_OK;
}

// ---- stationary -----------------------------------------------------------
mgc_status solve_stationary(mgc_grid g, void* u, const void* f, const mgc_solve_opts* o, mgc_stats* st) {
  double rr, ff;
  mgc_status rc = exact_residual(g, u, f, g->ws + g->r64, &rr, &ff);
  if (rc) return rc;
  const double fn = std::sqrt(ff);
  double rel = std::sqrt(rr) / fn;
  record(st, 0, rel);
  int it = 0;
  while (rel > o->tol && it < o->max_it && std::isfinite(rel)) {
    mgcccs_cycle<double>(g, u, f, false);
    ++it;
    rc = exact_residual(g, u, f, g->ws + g->r64, &rr, &ff);
    if (rc) return rc;
    rel = std::sqrt(rr) / fn;
    record(st, it, rel);
  }
  if (st) { st->iters = it; st->vcycles = it; st->relres = rel; }
  return finish_status(rel, o->tol);
}

// ---- iterative refinement ---------------------------------------------------
mgc_status solve_ir(mgc_grid g, void* u, const void* f, const mgc_solve_opts* o, mgc_stats* st) {
  const int n = g->d.n, pitch = g->lv[0].pitch;
  double rr, ff;
  void* r = g->ws + g->r64;
  mgc_status rc = exact_residual(g, u, f, r, &rr, &ff);
  if (rc) return rc;
  const double fn = std::sqrt(ff);
  double rel = std::sqrt(rr) / fn;
  record(st, 0, rel);
  int it = 0, cyc = 0;
  // sc[0] = s, (sc[2], sc[3]) = (1/s, 0): the complex coefficient at a
  // 16-byte boundary (scal is 256-byte aligned) for k_update's double2 load
  double* sc = g->at<double>(g->scal) + 8;
  double* nr = g->at<double>(g->scal);
  const double Nn = (double)(n - 1) * (n - 1);
  while (rel > o->tol && it < o->max_it && std::isfinite(rel)) {
    launch_ir_scale(g->stream, nr, Nn, sc);
    if (o->inner == MGC_FP32) {
      launch_scale_copy<double, float>(g->stream, n, pitch, pitch, r, sc, g->ws + g->f32);
      for (int c = 0; c < o->inner_cycles; ++c) mgcccs_cycle<float>(g, g->ws + g->u32, g->ws + g->f32, c == 0);
      launch_update<float>(g->stream, n, pitch, 0, g->ws + g->u32, 1, (const double2*)(sc + 2), (double2*)u);
    } else {
      launch_scale_copy<double, double>(g->stream, n, pitch, pitch, r, sc, g->ws + g->tw);
      for (int c = 0; c < o->inner_cycles; ++c) mgcccs_cycle<double>(g, g->ws + g->tz, g->ws + g->tw, c == 0);
      launch_update<double>(g->stream, n, pitch, 0, g->ws + g->tz, 1, (const double2*)(sc + 2), (double2*)u);
    }
    cyc += o->inner_cycles;
    ++it;
    rc = exact_residual(g, u, f, r, &rr, &ff);
    if (rc) return rc;
    rel = std::sqrt(rr) / fn;
    record(st, it, rel);
  }
  if (st) { st->iters = it; st->vcycles = cyc; st->relres = rel; }
  return finish_status(rel, o->tol);
}

// ---- FGMRES -------------------------------------------------------------------
// One FGMRES restart cycle of mm <= m steps enqueued on stream st: Arnoldi
// with the MG-CCCS preconditioner, device-side Givens bookkeeping, the small
// least-squares solve and the update of u.  No host synchronisation.  The
// cycle's start (beta, g) is already on the device: launch_gmres_begin after
// the first residual, launch_cycle_end after each cycle.
void enqueue_fgmres_cycle(mgc_grid g, void* u, const mgc_solve_opts* o, double tol_abs, int mm,
                          hipStream_t st) {
  const int n = g->d.n, pitch = g->lv[0].pitch, m = o->restart;
  const bool f32 = o->inner == MGC_FP32;
  const size_t fb = g->field_bytes(0, P64), fbz = g->field_bytes(0, f32 ? P32 : P64);
  const size_t stride64 = fb / 16, stridez = fbz / (f32 ? 8 : 16);
  GmresState gs = gmres_state(g);
  double2* W = g->at<double2>(g->W);
  char* Z = g->ws + g->Z[f32 ? P32 : P64];
  double* p0 = g->at<double>(g->apart);
  double* p1 = p0 + ARNOLDI_PART;
  double* p2 = p1 + ARNOLDI_PART;
  Level<double> EX = exact_level(g);
  hipStream_t saved = g->stream;
  g->stream = st;                           // the cycle drivers launch on g->stream
  g->kt.used = 0;
  g->kt.run = -1;
  const bool per_step = g->kt.which == MGC_KT_APPLY_DOT || g->kt.which == MGC_KT_AXPY;
  const double Nint = (double)(n - 1) * (n - 1);
  // threshold of the selective second Gram-Schmidt pass; MGC_REORTH_ETA > 1
  // forces the second pass in every step (a test of that path)
  const char* eta_env = std::getenv("MGC_REORTH_ETA");
  const double eta = eta_env && std::atof(eta_env) > 0 ? std::atof(eta_env) : REORTH_ETA;
  for (int j = 0; j < mm; ++j) {
    g->kt.open = per_step || j == 0;
    double2* Wj = W + (size_t)j * stride64;
    double2* Wn = W + (size_t)(j + 1) * stride64;
    char* Zj = Z + (size_t)j * fbz;
    // preconditioner on the normalised basis vector v_j = s_j W_j
    // algorithmic bytes: z (inner precision), J basis vectors, Y written
    const int ta = kt_slot(g, MGC_KT_APPLY_DOT, Nint * ((f32 ? 8.0 : 16.0) + 16.0 * (j + 1) + 16.0));
    if (f32) {
      // the FP32 cycle's input: W_j rounded to FP32 (by the previous step's
      // Gram-Schmidt passes for j > 0), scaled by s_j on the fly
      if (j == 0) launch_scale_copy<double, float>(st, n, pitch, pitch, Wj, nullptr, g->ws + g->f32);
      precondition<float>(g, Zj, g->ws + g->f32, gs.scale + j);
      kt_mark(g, st, ta, 0);
      launch_apply_dot<float>(st, EX, Zj, stride64, W, j + 1, Wn, p0);
    } else {
      precondition<double>(g, Zj, Wj, gs.scale + j);
      kt_mark(g, st, ta, 0);
      launch_apply_dot<double>(st, EX, Zj, stride64, W, j + 1, Wn, p0);
    }
    kt_mark(g, st, ta, 1);
    // classical Gram-Schmidt with a selective second pass, then the
    // Hessenberg column and its Givens rotation on the device
    // timed: the first pass (the second one runs only when needed)
    // J in, Y in/out (and its FP32 copy out with the FP32 cycle)
    float2* y32 = f32 ? (float2*)(g->ws + g->f32) : nullptr;
    const int tx = kt_slot(g, MGC_KT_AXPY, Nint * (16.0 * (j + 1) + 32.0 + (f32 ? 8.0 : 0.0)));
    kt_mark(g, st, tx, 0);
    launch_axpy_pass(st, n, pitch, stride64, W, j + 1, Wn, y32, p0, p1, gs);
    kt_mark(g, st, tx, 1);
    launch_reorth_step(st, n, pitch, stride64, W, j + 1, Wn, y32, p0, p1, p2, gs, m, mm, tol_abs, eta);
  }
  g->kt.open = true;
  if (f32) launch_update<float>(st, n, pitch, stridez, Z, mm, gs.upcoef, (double2*)u);
  else launch_update<double>(st, n, pitch, stridez, Z, mm, gs.upcoef, (double2*)u);
  g->stream = saved;
}

// report slot in the handle's scalars: ||r||^2, ||f||^2, steps used
constexpr int REPORT = 32;

// After a restart cycle: the true residual W_0 = f - A u of the new iterate
// (the next cycle's first basis vector), its norm and ||f|| into scal[0..1]
// and the Krylov state, the report the host reads (scal[REPORT..]) and the
// next cycle's start, in two launches.
void enqueue_cycle_end(mgc_grid g, const void* u, const void* f, int m, hipStream_t st) {
  GmresState gs = gmres_state(g);
  double* scal = g->at<double>(g->scal);
  double* part = g->at<double>(g->part);
  launch_stencil<double, double, double, double>(st, exact_level(g), u, f, g->at<double2>(g->W), 0, part,
                                                 Finish{});
  launch_cycle_end(st, g->d.n, part, scal, gs, m, scal + REPORT);
}

mgc_status solve_fgmres(mgc_grid g, void* u, const void* f, const mgc_solve_opts* o, mgc_stats* st) {
  const int m = o->restart;
  hipStream_t s = g->stream;
  GmresState gs = gmres_state(g);
  double2* W = g->at<double2>(g->W);
  if (g->basis_dirty) {
    // a failed solve may have left non-finite values outside the interior,
    // which the padded-array passes would pick up: start from zeros again
    HIPCHK(g, hipMemsetAsync(W, 0, (size_t)(g->d.max_restart + 1) * g->field_bytes(0, P64), s));
    g->basis_dirty = false;
  }
  // W_0 = f - A u  (||W_0||^2 lands in gs.nrm2 for the next cycle's start)
  double rr, ff;
  mgc_status rc = exact_residual(g, u, f, W, &rr, &ff, gs.nrm2);
  if (rc) return rc;
  launch_gmres_begin(s, gs, m);
  const double fn = std::sqrt(ff);
  double rel = std::sqrt(rr) / fn;
  record(st, 0, rel);
  int it = 0, rs = 0;
  const bool use_graph = std::getenv("MGC_NO_GRAPH") == nullptr;
  while (rel > o->tol && it < o->max_it && std::isfinite(rel)) {
    const int mm = std::min(m, o->max_it - it);
    // with a timer class selected, every KT_SAMPLE-th restart cycle (the
    // first included) runs with the timer's event nodes, the others without
    const bool timed = g->kt.which != MGC_KT_NONE && rs % KT_SAMPLE == 0;
    int kt_slots = 0;
    if (use_graph) {
      GraphCache& gc = timed || g->kt.which == MGC_KT_NONE ? g->graph : g->plain;
      const int want = timed ? g->kt.which : MGC_KT_NONE;
      if (!gc.exec || gc.u != u || gc.f != f || gc.m != m || gc.mm != mm || gc.inner != (int)o->inner ||
          gc.tol_abs != o->tol * fn || gc.kt != want) {
        if (gc.exec) { (void)hipGraphExecDestroy(gc.exec); gc.exec = nullptr; }
        const int sel = g->kt.which;
        g->kt.which = want;                // capture the untimed cycle without timer nodes
        hipGraph_t graph;
        hipError_t e = hipStreamBeginCapture(g->cap, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
          // the restart cycle, the true residual of the new iterate (the next
          // cycle's W_0), the report the host reads and the next start
          enqueue_fgmres_cycle(g, u, o, o->tol * fn, mm, g->cap);
          enqueue_cycle_end(g, u, f, m, g->cap);
          e = hipStreamEndCapture(g->cap, &graph);
        }
        g->kt.which = sel;
        HIPCHK(g, e);
        if (g->failed) {                   // a timer node could not be added
          (void)hipGraphDestroy(graph);
          return MGC_EHIP;
        }
        e = hipGraphInstantiate(&gc.exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        HIPCHK(g, e);
        gc.u = u; gc.f = f; gc.m = m; gc.mm = mm; gc.inner = (int)o->inner; gc.tol_abs = o->tol * fn;
        gc.kt = want;
        gc.kt_slots = timed ? g->kt.used : 0;
        gc.kt_bytes = g->kt.bytes;
        gc.kt_count = g->kt.count;
      }
      HIPCHK(g, hipGraphLaunch(gc.exec, s));
      kt_slots = gc.kt_slots;
    } else {
      const int sel = g->kt.which;
      if (!timed) g->kt.which = MGC_KT_NONE;
      enqueue_fgmres_cycle(g, u, o, o->tol * fn, mm, s);
      g->kt.which = sel;
      if (g->failed) return MGC_EHIP;
      kt_slots = timed ? g->kt.used : 0;
      enqueue_cycle_end(g, u, f, m, s);
    }
    // one read-back per restart cycle: ||r||^2, ||f||^2 and the steps used
    double rep[3];
    HIPCHK(g, hipMemcpyAsync(rep, g->at<double>(g->scal) + REPORT, sizeof(rep), hipMemcpyDeviceToHost, s));
    HIPCHK(g, hipStreamSynchronize(s));
    rr = rep[0];
    ff = rep[1];
    const int kused = (int)rep[2];
    if (kt_slots > 0)
      kt_harvest(g, kt_slots, use_graph ? g->graph.kt_bytes : g->kt.bytes,
                 use_graph ? g->graph.kt_count : g->kt.count);
    it += std::min(kused, mm);
    rel = std::sqrt(rr) / fn;
    record(st, ++rs, rel);
  }
  if (st) { st->iters = it; st->vcycles = it; st->relres = rel; }
  if (!std::isfinite(rel)) g->basis_dirty = true;
  return finish_status(rel, o->tol);
}

// ---- BiCGSTAB ---------------------------------------------------------------
// Vectors in the Krylov basis W: r, r~, p, v, s, t (FP64); p^, s^ in Z (the
// inner precision).  Scalars in scal[BICG ..], the per-iteration report
// (||r||^2, ||s||^2, converged) in scal[BICG + 16 ..].
constexpr int BICG = 64;
void enqueue_bicg_iteration(mgc_grid g, void* u, const mgc_solve_opts* o, double tol2, hipStream_t st) {
  const int n = g->d.n, pitch = g->lv[0].pitch;
  const bool f32 = o->inner == MGC_FP32;
  const size_t s64 = g->field_bytes(0, P64) / 16;
  double2* W = g->at<double2>(g->W);
  double2 *r = W, *rt = W + s64, *p = W + 2 * s64, *v = W + 3 * s64, *sv = W + 4 * s64, *t = W + 5 * s64;
  char* Z = g->ws + g->Z[f32 ? P32 : P64];
  const size_t fbz = g->field_bytes(0, f32 ? P32 : P64);
  void* ph = Z;
  void* sh = Z + fbz;
  double* bs = g->at<double>(g->scal) + BICG;
  double* rep = bs + 16;
  double* p0 = g->at<double>(g->apart);
  double* p1 = p0 + ARNOLDI_PART;
  double* p2 = p1 + ARNOLDI_PART;
  Level<double> EX = exact_level(g);
  hipStream_t saved = g->stream;
  g->stream = st;
  // with the FP32 cycle, the p and s passes also write their vector rounded
  // to FP32 into the cycle's input field
  float2* in32 = f32 ? (float2*)(g->ws + g->f32) : nullptr;
  auto apply_pc = [&](const double2* in, void* out) {
    if (f32) precondition<float>(g, out, in32);
    else precondition<double>(g, out, in);
  };
  launch_bicg_p(st, n, pitch, r, v, p, in32, bs);
  apply_pc(p, ph);
  if (f32) launch_apply_dot<float>(st, EX, ph, s64, rt, 1, v, p0);
  else launch_apply_dot<double>(st, EX, ph, s64, rt, 1, v, p0);
  launch_bicg_s(st, n, pitch, p0, bs, r, v, sv, in32, p1);
  apply_pc(sv, sh);
  if (f32) launch_apply_dot<float>(st, EX, sh, s64, sv, 1, t, p2);
  else launch_apply_dot<double>(st, EX, sh, s64, sv, 1, t, p2);
  if (f32) launch_bicg_x<float>(st, n, pitch, p2, p1, tol2, bs, ph, sh, sv, t, rt, r, (double2*)u, p0);
  else launch_bicg_x<double>(st, n, pitch, p2, p1, tol2, bs, ph, sh, sv, t, rt, r, (double2*)u, p0);
  launch_bicg_rho(st, n, p0, bs, rep);
  g->stream = saved;
}

mgc_status solve_bicgstab(mgc_grid g, void* u, const void* f, const mgc_solve_opts* o, mgc_stats* st) {
  if (g->d.max_restart < 5) return fail(MGC_EINVAL, "BiCGSTAB needs desc.max_restart >= 5");
  hipStream_t s = g->stream;
  const size_t fb = g->field_bytes(0, P64);
  double2* W = g->at<double2>(g->W);
  if (g->basis_dirty) {
    HIPCHK(g, hipMemsetAsync(W, 0, (size_t)(g->d.max_restart + 1) * fb, s));
    g->basis_dirty = false;
  }
  double* bs = g->at<double>(g->scal) + BICG;
  double rr, ff;
  mgc_status rc = exact_residual(g, u, f, W, &rr, &ff);        // r = f - A u
  if (rc) return rc;
  const double fn = std::sqrt(ff);
  double rel = std::sqrt(rr) / fn;
  record(st, 0, rel);
  // r~ = r, p = v = 0, scalars from ||r||^2
  HIPCHK(g, hipMemcpyAsync(W + fb / 16, W, fb, hipMemcpyDeviceToDevice, s));
  launch_fill_zero(s, W + 2 * (fb / 16), 2 * fb);
  launch_bicg_init(s, bs, g->at<double>(g->scal));
  HIPCHK(g, hipGetLastError());
  const double tol2 = (o->tol * fn) * (o->tol * fn);
  const bool use_graph = std::getenv("MGC_NO_GRAPH") == nullptr;
  int it = 0;
  bool conv = false;
  while (rel > o->tol && !conv && it < o->max_it && std::isfinite(rel)) {
    if (use_graph) {
      GraphCache& gc = g->bicg_graph;
      if (!gc.exec || gc.u != u || gc.f != f || gc.inner != (int)o->inner || gc.tol_abs != tol2) {
        if (gc.exec) { (void)hipGraphExecDestroy(gc.exec); gc.exec = nullptr; }
        hipGraph_t graph;
        HIPCHK(g, hipStreamBeginCapture(g->cap, hipStreamCaptureModeThreadLocal));
        enqueue_bicg_iteration(g, u, o, tol2, g->cap);
        HIPCHK(g, hipStreamEndCapture(g->cap, &graph));
        hipError_t e = hipGraphInstantiate(&gc.exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        HIPCHK(g, e);
        gc.u = u; gc.f = f; gc.inner = (int)o->inner; gc.tol_abs = tol2;
      }
      HIPCHK(g, hipGraphLaunch(gc.exec, s));
    } else {
      enqueue_bicg_iteration(g, u, o, tol2, s);
      HIPCHK(g, hipGetLastError());
    }
    double rep[3];
    HIPCHK(g, hipMemcpyAsync(rep, bs + 16, sizeof(rep), hipMemcpyDeviceToHost, s));
    HIPCHK(g, hipStreamSynchronize(s));
    ++it;
    conv = rep[2] != 0.0;
    rel = std::sqrt(conv ? rep[1] : rep[0]) / fn;
    record(st, it, rel);
  }
  rc = exact_residual(g, u, f, g->ws + g->r64, &rr, &ff);
  if (rc) return rc;
  rel = std::sqrt(rr) / fn;
  if (st) { st->iters = it; st->vcycles = 2 * it; st->relres = rel; }
  if (!std::isfinite(rel)) g->basis_dirty = true;
  return finish_status(rel, o->tol);
}

}  // namespace

namespace {
// ----------------------------------------------------------------------------
// Test functions of eq. testfunction with forward-mode derivatives in Z1.
struct Dual {
  double v, d;
};
inline Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
inline Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
inline Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
inline Dual operator/(Dual a, Dual b) { return {a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v)}; }
inline Dual dsqrt(Dual a) {
  const double s = std::sqrt(a.v);
  return {s, 0.5 * a.d / s};
}
inline Dual cst(double x) { return {x, 0.0}; }

// Regular solution of (-1/2 d2/dx2 - Z1/x - k^2/2) phi = 0 by the 3-point
// recurrence on the real nodes, scaled to local amplitude 1/sqrt(p) at R0,
// p = sqrt(k^2 - 2 V1(R0)); out[j] = t_j phi(x_j) with trapezoid weights t
// (h, h/2 at j0) for 1 <= j <= min(j0, n-1), zero elsewhere; dout = d out / d Z1.
// With `tab` (the potential at the real nodes, any model) the potential comes
// from the table and the derivative part is zero.
void test_function(const Axis& ax, double Z1, double k, std::vector<double>& out,
                   std::vector<double>& dout, const std::vector<double>* tab = nullptr) {
  const int n = ax.n, j0 = ax.j0;
  const double h = ax.h;
  const Dual z1 = {Z1, 1.0};
  const int top = std::min(j0 + 1, n);
  std::vector<Dual> ph(top + 1, cst(0.0));
  ph[1] = cst(h);
  for (int j = 1; j < top; ++j) {
    const Dual V1 = tab ? cst((*tab)[j]) : cst(0.0) - z1 / cst(j * h);
    ph[j + 1] = cst(2.0) * ph[j] - ph[j - 1] + cst(2.0 * h * h) * (V1 - cst(0.5 * k * k)) * ph[j];
  }
  const int jr = std::min(j0, top - 1);
  const Dual p = dsqrt(cst(k * k) - cst(2.0) * (tab ? cst((*tab)[jr]) : cst(0.0) - z1 / cst(jr * h)));
  const Dual dphi = (ph[jr + 1] - ph[jr - 1]) / cst(2.0 * h);
  const Dual q = dphi / p;
  const Dual amp = dsqrt(ph[jr] * ph[jr] + q * q);
  const Dual sc = cst(1.0) / (amp * dsqrt(p));
  out.assign(n + 1, 0.0);
  dout.assign(n + 1, 0.0);
  for (int j = 1; j <= std::min(j0, n - 1); ++j) {
    const double t = (j == j0 ? 0.5 * h : h);
    const Dual v = ph[j] * sc;
    out[j] = t * v.v;
    dout[j] = t * v.d;
  }
}

// k0^2 of the cross-section prefactor: twice the energy of the incoming
// electron over the target's ground state (Temkin-Poet: E + Z1^2 / 2; a
// general model: E minus the lowest x1 bound state of the exact axis).
double k0sq_of(mgc_grid g) {
  return g->pot.kind == POT_TP ? 2.0 * (g->E + 0.5 * g->Z1 * g->Z1) : 2.0 * (g->E - g->lam1x);
}
// The amplitude source chi - V12 u: for the Temkin-Poet form the kernels take
// (tm, chi) as they are; for a general two-body table the source is formed in
// r64 first and V12 is replaced by the zero table.
void amp_source(mgc_grid g, hipStream_t st, const void* u, const void*& chi, const double2*& tm) {
  if (g->pot.kind == POT_TP) {
    tm = exact_level(g).tm;
    return;
  }
  double2* s = g->at<double2>(g->r64);
  launch_src_v12(st, g->d.n, g->lv[0].pitch, static_cast<const double2*>(chi), exact_level(g).v12,
                 static_cast<const double2*>(u), s);
  chi = s;
  tm = g->at<const double2>(g->tm0);
}

}  // namespace

// ============================================================================
extern "C" {

const char* mgc_last_error(void) { return g_err.c_str(); }

mgc_status mgc_create_grid(const mgc_grid_desc* d, void* hip_stream, mgc_grid* out) {
  if (!d || !out) return fail(MGC_EINVAL, "null argument");
  *out = nullptr;
  const int n = d->n;
  if (n < 8 || (n & (n - 1))) return fail(MGC_EINVAL, "n must be a power of two >= 8");
  if (n > 16384) return fail(MGC_EINVAL, "n too large");
  if (!(d->L > 0) || !(d->R0 > 0) || !(d->R0 <= d->L)) return fail(MGC_EINVAL, "need 0 < R0 <= L");
  if (!(d->theta > 0) || !(d->theta < M_PI / 2)) return fail(MGC_EINVAL, "theta must lie in (0, pi/2)");
  if (d->levels < 1 || (n >> (d->levels - 1)) < 4) return fail(MGC_EINVAL, "too many levels");
  const int nc = n >> (d->levels - 1);
  if ((nc - 1) * (nc - 1) > 1024) return fail(MGC_EINVAL, "coarsest level holds more than 1024 unknowns");
  const double hc = d->L / nc;
  const double jc = d->R0 / hc;
  if (std::abs(jc - std::round(jc)) > 1e-9 * std::max(1.0, jc)) return fail(MGC_EINVAL, "R0 must be a node of the coarsest level");
  if (d->M < 0 || d->Lch < 0 || d->M > 16 || d->Lch > 16) return fail(MGC_EINVAL, "channel counts must lie in [0, 16]");
  if ((d->M == 0) != (d->Lch == 0)) return fail(MGC_EINVAL, "M and Lch must both be zero or both positive");
  if (d->M >= n - 1 || d->Lch >= n - 1) return fail(MGC_EINVAL, "too many channels for the grid");
  if (!(d->omega > 0) || !(d->omega < 2)) return fail(MGC_EINVAL, "omega must lie in (0, 2)");
  if (d->nu1 < 0 || d->nu2 < 0 || d->nu1 + d->nu2 < 1 || d->nu1 > 8 || d->nu2 > 8) return fail(MGC_EINVAL, "bad smoothing counts");
  if (!(d->pc_gamma >= 0) || !(d->pc_gamma < M_PI / 4)) return fail(MGC_EINVAL, "pc_gamma must lie in [0, pi/4)");
  if (!(d->pc_gamma0 >= 0) || !(d->pc_gamma0 < M_PI / 4)) return fail(MGC_EINVAL, "pc_gamma0 must lie in [0, pi/4)");
  if (!(d->gamma >= 0) || !(d->gamma < M_PI / 4)) return fail(MGC_EINVAL, "gamma must lie in [0, pi/4)");
  if (d->pc_first_level < 0) return fail(MGC_EINVAL, "pc_first_level must be >= 0");
  if (d->smoother != MGC_SMOOTH_JACOBI && d->smoother != MGC_SMOOTH_GMRES3)
    return fail(MGC_EINVAL, "smoother must be MGC_SMOOTH_JACOBI or MGC_SMOOTH_GMRES3");
  if (d->gs_from < 0 || d->gs_from > d->levels) return fail(MGC_EINVAL, "gs_from must lie in [0, levels]");
  if (d->pc_order != MGC_PC_MG_CCCS && d->pc_order != MGC_PC_DEFLATION)
    return fail(MGC_EINVAL, "pc_order must be MGC_PC_MG_CCCS or MGC_PC_DEFLATION");
  if (d->max_restart < 0 || d->max_restart > MGC_MAX_RESTART)
    return fail(MGC_EINVAL, "max_restart must lie in [0, 16]");
  if ((d->precisions & 1) == 0 || (d->precisions & ~3)) return fail(MGC_EINVAL, "precisions must include MGC_FP64");

  mgc_grid g = new mgc_grid_s();
  g->d = *d;
  g->stream = (hipStream_t)hip_stream;
  if (hipGetDevice(&g->device) != hipSuccess) g->device = 0;
  if (hipStreamCreateWithFlags(&g->cap, hipStreamNonBlocking) != hipSuccess) {
    delete g;
    return fail(MGC_EHIP, "could not create the capture stream");
  }
  g->prec_on[P64] = true;
  g->prec_on[P32] = (d->precisions & 2) != 0;
  g->exact = make_axis(n, d->L, d->R0, d->theta, d->gamma);
  for (int l = 0; l < d->levels; ++l) {
    LevelInfo L;
    L.n = n >> l;
    L.pitch = pitch_for(L.n);
    const double gam = (l >= d->pc_first_level) ? d->pc_gamma : d->pc_gamma0;
    L.ax = make_axis(L.n, d->L, d->R0, d->theta, gam);
    g->lv.push_back(L);
  }
  const int N = n - 1;
  // SPIKE chunks: the chunk chains are sequential in the rows of a chunk,
  // the interface system is one precomputed matrix applied in parallel, so
  // the chunks are kept short (about sqrt(2N) of them); at most 64, the bound
  // the interface mat-vec stages in LDS ((P-1) 2M <= 63 x 32 entries)
  auto chunks = [&](int) {
    int P = (int)std::lround(std::sqrt(2.0 * N));
    return std::max(1, std::min(64, P));
  };
  g->PA = chunks(d->M);
  g->PB = chunks(d->Lch);
  g->nchunksB = (N + 63) / 64;
  layout(g);
  *out = g;
  return MGC_OK;
}

mgc_status mgc_set_schedule(mgc_grid g, const mgc_schedule* s) {
  if (!g || !s) return fail(MGC_EINVAL, "null argument");
  if (s->small_tiles < -1) return fail(MGC_EINVAL, "small_tiles must be -1 or a level bit mask");
  if ((s->level_pairs != 0 && s->level_pairs != 1) || (s->coarse_tail != 0 && s->coarse_tail != 1))
    return fail(MGC_EINVAL, "level_pairs and coarse_tail must be 0 or 1");
  g->sched = *s;
  drop_graph(g);                           // the captured restart cycle has the old launches
  return MGC_OK;
}

mgc_status mgc_get_schedule(mgc_grid g, mgc_schedule* s) {
  if (!g || !s) return fail(MGC_EINVAL, "null argument");
  *s = g->sched;
  return MGC_OK;
}

mgc_status mgc_workspace_bytes(mgc_grid g, size_t* bytes) {
  if (!g || !bytes) return fail(MGC_EINVAL, "null argument");
  *bytes = g->need;
  return MGC_OK;
}

mgc_status mgc_bind_workspace(mgc_grid g, void* ptr, size_t bytes) {
  if (!g) return fail(MGC_EINVAL, "null handle");
  if (g->failed) return fail(MGC_ESTATE, "handle failed");
  if (!ptr || ((uintptr_t)ptr & 255)) return fail(MGC_EINVAL, "workspace must be non-null and 256-byte aligned");
  if (bytes < g->need) return fail(MGC_ENOMEM, "workspace too small");
  g->ws = (char*)ptr;
  g->ws_bytes = bytes;
  HIPCHK(g, hipMemsetAsync(g->ws, 0, g->need, g->stream));
  // exact-operator dual weights (for the transpose solve)
  mgc_status rc = upload_cplx<double>(g, g->exact_w, g->exact.w);
  if (rc) return rc;
  if ((rc = upload_cplx<double>(g, g->exact_z, g->exact.z))) return rc;
  g->have_pot = g->have_energy = false;
  return MGC_OK;
}

mgc_status mgc_field_pitch(mgc_grid g, int level, int* pitch) {
  if (!g || !pitch) return fail(MGC_EINVAL, "null argument");
  if (level < 0 || level >= (int)g->lv.size()) return fail(MGC_EINVAL, "level out of range");
  *pitch = g->lv[level].pitch;
  return MGC_OK;
}

}  // extern "C"

namespace {
// Tables and bound states of the model in g->pot (shared by both set_potential
// entry points).
mgc_status apply_potential(mgc_grid g) {
  auto t0 = std::chrono::steady_clock::now();
  drop_graph(g);
  g->have_pot = g->have_energy = false;
  g->si_count = 0;
  const PotModel& pm = g->pot;
  const int n = g->d.n, M = g->d.M, Lc = g->d.Lch;
  mgc_status rc;
  std::string err;
  // level tables of the exact operator and of the hierarchy
  {
    auto t = level_tables(g->exact, pm);
    if ((rc = upload_cplx<double>(g, g->exact_tab, t))) return rc;
    if (g->prec_on[P32] && (rc = upload_cplx<float>(g, g->exact_tab32, t))) return rc;
    if (pm.kind == POT_EXP) {
      auto v = two_body_table(g->exact, pm, g->lv[0].pitch);
      if ((rc = upload_cplx<double>(g, g->exact_v12[P64], v))) return rc;
      if (g->prec_on[P32] && (rc = upload_cplx<float>(g, g->exact_v12[P32], v))) return rc;
    }
  }
  for (size_t l = 0; l < g->lv.size(); ++l) {
    auto t = level_tables(g->lv[l].ax, pm);
    if ((rc = upload_cplx<double>(g, g->lv[l].tab[P64], t))) return rc;
    if (g->prec_on[P32] && (rc = upload_cplx<float>(g, g->lv[l].tab[P32], t))) return rc;
    if (pm.kind == POT_EXP) {
      auto v = two_body_table(g->lv[l].ax, pm, g->lv[l].pitch);
      if ((rc = upload_cplx<double>(g, g->lv[l].v12[P64], v))) return rc;
      if (g->prec_on[P32] && (rc = upload_cplx<float>(g, g->lv[l].v12[P32], v))) return rc;
    }
  }
  // the x1 potential at the real nodes of the exact axis (test functions of
  // the amplitudes) and the zero table that stands for V12 once the source
  // chi - V12 u has been formed with a general two-body table
  {
    const Axis& ex = g->exact;
    g->v1r_host.assign(n + 1, 0.0);
    for (int j = 1; j <= n; ++j) {
      const double x = (double)j * ex.h;
      g->v1r_host[j] = pm.kind == POT_TP ? 0.0 - pm.Z1 / x : -pm.a1 * std::exp(-pm.b1 * x * x);
    }
    if ((rc = upload(g, g->v1r, g->v1r_host.data(), (n + 1) * sizeof(double)))) return rc;
    if ((rc = upload_cplx<double>(g, g->tm0, std::vector<cd>(n + 1, 0.0)))) return rc;
    g->lam1x = -0.5 * pm.Z1 * pm.Z1;
    if (pm.kind == POT_EXP) {
      std::vector<cd> l1;
      std::vector<std::vector<cd>> p1;
      if (!bound_states(ex, one_body(ex, pm, 1), 1, 2, l1, p1, err)) return fail(MGC_ENUMERIC, err);
      g->lam1x = l1[0].real();
    }
  }
  // bound states of the hierarchy's level-0 one-body Hamiltonians
  const Axis& ax = g->lv[0].ax;
  if (M > 0) {
    if (!bound_states(ax, one_body(ax, pm, 1), M, 2, g->lamA, g->phi, err)) return fail(MGC_ENUMERIC, err);
    if (!bound_states(ax, one_body(ax, pm, 2), Lc, 2, g->lamB, g->vphi, err)) return fail(MGC_ENUMERIC, err);
    std::vector<cd> wphi((size_t)M * (n + 1)), phi((size_t)M * (n + 1)),
        wvphi((size_t)Lc * (n + 1)), vphi((size_t)Lc * (n + 1));
    for (int i = 0; i < M; ++i)
      for (int j = 0; j <= n; ++j) {
        phi[(size_t)i * (n + 1) + j] = g->phi[i][j];
        wphi[(size_t)i * (n + 1) + j] = ax.w[j] * g->phi[i][j];
      }
    for (int l = 0; l < Lc; ++l)
      for (int k = 0; k <= n; ++k) {
        vphi[(size_t)l * (n + 1) + k] = g->vphi[l][k];
        wvphi[(size_t)l * (n + 1) + k] = ax.w[k] * g->vphi[l][k];
      }
    for (int p = 0; p < 2; ++p) {
      if (!g->prec_on[p]) continue;
      const CcOff& c = g->cc[p];
      auto up = [&](size_t off, const std::vector<cd>& v) {
        return p == P64 ? upload_cplx<double>(g, off, v) : upload_cplx<float>(g, off, v);
      };
      if ((rc = up(c.wphi, wphi)) || (rc = up(c.phi, phi)) || (rc = up(c.wvphi, wvphi)) ||
          (rc = up(c.vphi, vphi)))
        return rc;
    }
  }
  g->have_pot = true;
  g->t_setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return MGC_OK;
}
}  // namespace

extern "C" {

mgc_status mgc_set_potential(mgc_grid g, double Z1, double Z2, double lambda) {
  mgc_status rc = check_ready(g, false);
  if (rc) return rc;
  if (!std::isfinite(Z1) || !std::isfinite(Z2) || !std::isfinite(lambda) || Z1 < 0)
    return fail(MGC_EINVAL, "potential strengths must be finite, Z1 >= 0");
  g->Z1 = Z1; g->Z2 = Z2; g->lam = lambda;
  g->pot = PotModel();
  g->pot.Z1 = Z1; g->pot.Z2 = Z2; g->pot.lam = lambda;
  return apply_potential(g);
}

mgc_status mgc_set_potential_exp(mgc_grid g, double a1, double b1, double a2, double b2, double c12, double d12) {
  mgc_status rc = check_ready(g, false);
  if (rc) return rc;
  for (double v : {a1, b1, a2, b2, c12, d12})
    if (!std::isfinite(v)) return fail(MGC_EINVAL, "exponential model parameters must be finite");
  if (b1 < 0 || b2 < 0 || d12 < 0) return fail(MGC_EINVAL, "exponential model decay rates must be >= 0");
  if (!g->d.pot_tables)
    return fail(MGC_EINVAL, "the exponential model needs a handle created with pot_tables = 1");
  g->pot = PotModel();
  g->pot.kind = POT_EXP;
  g->pot.a1 = a1; g->pot.b1 = b1; g->pot.a2 = a2; g->pot.b2 = b2; g->pot.c12 = c12; g->pot.d12 = d12;
  g->Z1 = g->Z2 = g->lam = 0;
  return apply_potential(g);
}

mgc_status mgc_channel_energies(mgc_grid g, double* lamA, double* lamB) {
  mgc_status rc = check_ready(g, false);
  if (rc) return rc;
  if (!g->have_pot) return fail(MGC_ESTATE, "set_potential required");
  for (int i = 0; i < g->d.M && lamA; ++i) { lamA[2 * i] = g->lamA[i].real(); lamA[2 * i + 1] = g->lamA[i].imag(); }
  for (int l = 0; l < g->d.Lch && lamB; ++l) { lamB[2 * l] = g->lamB[l].real(); lamB[2 * l + 1] = g->lamB[l].imag(); }
  return MGC_OK;
}

}  // extern "C"


namespace {
// Channel potential V[node][i][m] = sum_j w_j (lam / z_max(j,node)) f_i(j) f_m(j)
// evaluated with prefix sums:  (lam/z_node) sum_{j<=node} g_im(j) + sum_{j>node} (lam/z_j) g_im(j).
std::vector<cd> channel_potential(const Axis& ax, double lam, const std::vector<std::vector<cd>>& f) {
  const int n = ax.n, M = (int)f.size(), MM = M * M;
  std::vector<cd> V((size_t)(n + 1) * MM, 0.0), pre(MM, 0.0), suf((size_t)(n + 2) * MM, 0.0);
  for (int j = n - 1; j >= 1; --j)
    for (int i = 0; i < M; ++i)
      for (int m = 0; m < M; ++m)
        suf[(size_t)j * MM + i * M + m] = suf[(size_t)(j + 1) * MM + i * M + m] +
                                          (lam / ax.z[j]) * ax.w[j] * f[i][j] * f[m][j];
  for (int k = 1; k < n; ++k) {
    for (int i = 0; i < M; ++i)
      for (int m = 0; m < M; ++m) pre[i * M + m] += ax.w[k] * f[i][k] * f[m][k];
    for (int q = 0; q < MM; ++q)
      V[(size_t)k * MM + q] = (lam / ax.z[k]) * pre[q] + suf[(size_t)(k + 1) * MM + q];
  }
  return V;
}

// Channel potential of a general (symmetric) two-body model, summed directly:
// V[node][i][m] = sum_j w_j V12(z_j, z_node) f_i(j) f_m(j).
std::vector<cd> channel_potential(const Axis& ax, const PotModel& pm, const std::vector<std::vector<cd>>& f) {
  const int n = ax.n, M = (int)f.size(), MM = M * M;
  std::vector<cd> V((size_t)(n + 1) * MM, 0.0), G((size_t)(n + 1) * MM, 0.0);
  for (int j = 1; j < n; ++j)
    for (int i = 0; i < M; ++i)
      for (int m = 0; m < M; ++m) G[(size_t)j * MM + i * M + m] = ax.w[j] * f[i][j] * f[m][j];
  for (int k = 1; k < n; ++k) {
    cd* out = &V[(size_t)k * MM];
    for (int j = 1; j < n; ++j) {
      const cd v = pm.v12(ax, j, k);
      const cd* gj = &G[(size_t)j * MM];
      for (int q = 0; q < MM; ++q) out[q] += v * gj[q];
    }
  }
  return V;
}

template <typename T>
mgc_status upload_factors(mgc_grid g, int p, const SysOff& so, const ChannelFactors& f) {
  mgc_status rc;
  auto up = [&](size_t off, const std::vector<cd>& v) { return upload_cplx<T>(g, off, v); };
  if ((rc = up(so.G, f.G)) || (rc = up(so.Vs, f.Vs)) || (rc = up(so.Ws, f.Ws)) || (rc = up(so.lo, f.lo)) ||
      (rc = up(so.up, f.up)))
    return rc;
  if (f.P > 1) {
    if ((rc = up(so.Rinv, f.Rinv)) || (rc = up(so.Tif, f.Tif)))
      return rc;
  }
  (void)p;
  return upload(g, so.start, f.start.data(), f.start.size() * sizeof(int));
}
}  // namespace

extern "C" {

mgc_status mgc_set_energy(mgc_grid g, double E) {
  mgc_status rc = check_ready(g, false);
  if (rc) return rc;
  if (!g->have_pot) return fail(MGC_ESTATE, "set_potential required before set_energy");
  if (!std::isfinite(E)) return fail(MGC_EINVAL, "E must be finite");
  auto t0 = std::chrono::steady_clock::now();
  drop_graph(g);
  g->have_energy = false;
  g->E = E;
  std::string err;
  const int n = g->d.n, N = n - 1, M = g->d.M, Lc = g->d.Lch;
  // coupled channel systems on the hierarchy's level-0 axis
  if (M > 0) {
    const Axis& ax = g->lv[0].ax;
    for (int sys = 0; sys < 2; ++sys) {
      const bool isA = sys == 0;
      const int m = isA ? M : Lc;
      const auto& basis = isA ? g->phi : g->vphi;
      const auto& lamv = isA ? g->lamA : g->lamB;
      // one-body potential of the free coordinate (x2 for the A system)
      const std::vector<cd> Vo = one_body(ax, g->pot, isA ? 2 : 1);
      std::vector<cd> V = g->pot.kind == POT_TP ? channel_potential(ax, g->lam, basis)
                                                : channel_potential(ax, g->pot, basis);
      std::vector<cd> lo(N), upv(N), D((size_t)N * m * m, 0.0);
      for (int t = 0; t < N; ++t) {
        const int node = t + 1;
        lo[t] = ax.a[node];
        upv[t] = ax.c[node];
        for (int q = 0; q < m * m; ++q) D[(size_t)t * m * m + q] = V[(size_t)node * m * m + q];
        const cd dd = ax.b[node] + Vo[node] - E;
        for (int i = 0; i < m; ++i) D[(size_t)t * m * m + i * m + i] += dd + lamv[i];
      }
      ChannelFactors f;
      if (!factor_channels(N, m, isA ? g->PA : g->PB, lo, upv, D, f, err)) return fail(MGC_ENUMERIC, err);
      if ((rc = upload_factors<double>(g, P64, isA ? g->cc[P64].A : g->cc[P64].B, f))) return rc;
      if (g->prec_on[P32] && (rc = upload_factors<float>(g, P32, isA ? g->cc[P32].A : g->cc[P32].B, f)))
        return rc;
    }
  }
  // coarsest level: dense inverse of the rediscretised operator
  {
    const LevelInfo& C = g->lv.back();
    const int nc = C.n, m = nc - 1, Nc = m * m;
    const Axis& ax = C.ax;
    std::vector<cd> A((size_t)Nc * Nc, 0.0);
    for (int k = 1; k < nc; ++k)
      for (int j = 1; j < nc; ++j) {
        const int r = (k - 1) * m + (j - 1);
        const cd d = ax.b[j] + g->pot.v1(ax.z[j]) + ax.b[k] + g->pot.v2(ax.z[k]) + g->pot.v12(ax, j, k) - E;
        A[(size_t)r * Nc + r] = d;
        if (j > 1) A[(size_t)r * Nc + r - 1] = ax.a[j];
        if (j < m) A[(size_t)r * Nc + r + 1] = ax.c[j];
        if (k > 1) A[(size_t)r * Nc + r - m] = ax.a[k];
        if (k < m) A[(size_t)r * Nc + r + m] = ax.c[k];
      }
    std::vector<cd> inv;
    if (!dense_inverse(Nc, A, inv, err)) return fail(MGC_ENUMERIC, "coarsest operator: " + err);
    if ((rc = upload_cplx<double>(g, g->coarse_inv, inv))) return rc;
  }
  g->have_energy = true;
  g->t_setup_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return MGC_OK;
}

mgc_status mgc_build_rhs_tp(mgc_grid g, void* chi, mgc_precision prec) {
  mgc_status rc = check_ready(g, false);
  if (rc) return rc;
  if (g->pot.kind != POT_TP) return fail(MGC_EINVAL, "defined for the Temkin-Poet model only");
  if (!g->have_pot) return fail(MGC_ESTATE, "set_potential required");
  if (!chi) return fail(MGC_EINVAL, "null field");
  if (prec != MGC_FP64) return fail(MGC_EINVAL, "right-hand side is built in FP64");
  if (!(g->E + 0.5 * g->Z1 * g->Z1 > 0))
    return fail(MGC_EINVAL, "impact right-hand side needs E above the 1s threshold -Z1^2/2");
  const double k0 = std::sqrt(2.0 * (g->E + 0.5 * g->Z1 * g->Z1));
  launch_rhs_tp(g->stream, g->d.n, g->lv[0].pitch, g->exact.j0, g->at<const double2>(g->exact_z), g->Z1, g->Z2,
                g->lam, k0, (double2*)chi);
  HIPCHK(g, hipGetLastError());
  HIPCHK(g, hipStreamSynchronize(g->stream));
  return MGC_OK;
}

mgc_status mgc_residual(mgc_grid g, const void* u, const void* f, void* r, double* relres, mgc_precision prec) {
  mgc_status rc = check_ready(g);
  if (rc) return rc;
  if (!u || !f || !r || r == u) return fail(MGC_EINVAL, "bad field pointers");
  if (prec == MGC_FP64) {
    if (relres) {
      double rr, ff;
      if ((rc = exact_residual(g, u, f, r, &rr, &ff))) return rc;
      *relres = std::sqrt(rr / ff);
    } else {
      launch_stencil<double, double, double, double>(g->stream, exact_level(g), u, f, r, 0, nullptr);
    }
  } else {
    if (!g->prec_on[P32]) return fail(MGC_EINVAL, "FP32 not enabled in the descriptor");
    double* part = g->at<double>(g->part);
    launch_stencil<float, float, float, float>(g->stream, exact_level<float>(g), u, f, r, 0, relres ? part : nullptr);
    if (relres) {
      double* out = g->at<double>(g->scal);
      launch_sum_partials(g->stream, launch_stencil_blocks(g->d.n), 2, part, out);
      double h[2];
      HIPCHK(g, hipMemcpyAsync(h, out, sizeof(h), hipMemcpyDeviceToHost, g->stream));
      HIPCHK(g, hipStreamSynchronize(g->stream));
      *relres = std::sqrt(h[0] / h[1]);
    }
  }
  HIPCHK(g, hipGetLastError());
  return MGC_OK;
}

mgc_status mgc_vcycle(mgc_grid g, void* u, const void* f, mgc_precision prec) {
  mgc_status rc = check_ready(g);
  if (rc) return rc;
  if (!u || !f || u == f) return fail(MGC_EINVAL, "bad field pointers");
  if (prec == MGC_FP64) vcycle_level<double>(g, 0, u, f, false);
  else if (g->prec_on[P32]) vcycle_level<float>(g, 0, u, f, false);
  else return fail(MGC_EINVAL, "FP32 not enabled in the descriptor");
  HIPCHK(g, hipGetLastError());
  return MGC_OK;
}

mgc_status mgc_cccs(mgc_grid g, void* u, const void* f, mgc_precision prec) {
  mgc_status rc = check_ready(g);
  if (rc) return rc;
  if (!u || !f || u == f) return fail(MGC_EINVAL, "bad field pointers");
  if (prec == MGC_FP64) cccs_apply<double>(g, u, f);
  else if (g->prec_on[P32]) cccs_apply<float>(g, u, f);
  else return fail(MGC_EINVAL, "FP32 not enabled in the descriptor");
  HIPCHK(g, hipGetLastError());
  return MGC_OK;
}

}  // extern "C"

namespace mgc {
// mgc_cccs with its scratch (partials, channel vectors) at `scratch`, a
// device buffer of `bytes` bytes (the no-allocation entry point passes the
// library's static array); the region used is cleared first by a fill
// kernel.  MGC_EINVAL if it does not fit.
mgc_status cccs_with_scratch(mgc_grid g, void* u, const void* f, mgc_precision prec, void* scratch, size_t bytes) {
  mgc_status rc = check_ready(g);
  if (rc) return rc;
  if (!u || !f || u == f) return fail(MGC_EINVAL, "bad field pointers");
  if (prec != MGC_FP64 && !g->prec_on[P32]) return fail(MGC_EINVAL, "FP32 not enabled in the descriptor");
  if (g->d.M == 0 && g->d.Lch == 0) return MGC_OK;
  const int p = prec == MGC_FP64 ? P64 : P32;
  size_t off = 0;
  auto take = [&](size_t b) {
    size_t o = off;
    off = align256(off + b);
    return o;
  };
  CcOff c;
  cccs_scratch_layout(g, p, take, c);
  if (off > bytes)
    return fail(MGC_EINVAL, "CCCS scratch of this grid (" + std::to_string(off) + " bytes) exceeds the " +
                                std::to_string(bytes) + "-byte static scratch");
  launch_fill_zero(g->stream, scratch, off);
  const CccsScratch w = scratch_at(static_cast<char*>(scratch), c);
  if (p == P64) cccs_apply<double>(g, u, f, nullptr, &w);
  else cccs_apply<float>(g, u, f, nullptr, &w);
  HIPCHK(g, hipGetLastError());
  return MGC_OK;
}
int handle_device(mgc_grid g) { return g->device; }
mgc_status set_error(mgc_status s, const char* msg) { return fail(s, msg); }
}  // namespace mgc

extern "C" {

static mgc_status validate_opts(mgc_grid g, const mgc_solve_opts* o) {
  if (!o) return fail(MGC_EINVAL, "null options");
  if (!(o->tol > 0) || o->max_it < 1) return fail(MGC_EINVAL, "need tol > 0 and max_it >= 1");
  if (o->inner != MGC_FP64 && o->inner != MGC_FP32) return fail(MGC_EINVAL, "bad inner precision");
  if (o->inner == MGC_FP32 && !g->prec_on[P32]) return fail(MGC_EINVAL, "FP32 not enabled in the descriptor");
  switch (o->outer) {
    case MGC_STATIONARY:
      if (o->inner != MGC_FP64) return fail(MGC_EINVAL, "stationary iteration runs in FP64");
      if ((g->d.pc_first_level == 0 ? g->d.pc_gamma : g->d.pc_gamma0) != g->d.gamma)
        return fail(MGC_EINVAL, "stationary iteration needs the exact level-0 operator (level 0 on the system's contour)");
      break;
    case MGC_IR:
      if (o->inner_cycles < 1 || o->inner_cycles > 16) return fail(MGC_EINVAL, "inner_cycles must lie in [1, 16]");
      break;
    case MGC_FGMRES:
      if (o->restart < 1 || o->restart > g->d.max_restart) return fail(MGC_EINVAL, "restart must lie in [1, max_restart]");
      break;
    case MGC_BICGSTAB:
      if (g->d.max_restart < 5) return fail(MGC_EINVAL, "BiCGSTAB needs desc.max_restart >= 5");
      break;
    default:
      return fail(MGC_EINVAL, "bad outer method");
  }
  return MGC_OK;
}

mgc_status mgc_solve(mgc_grid g, void* u, const void* f, const mgc_solve_opts* o, mgc_stats* st) {
  mgc_status rc = check_ready(g);
  if (rc) return rc;
  if (!u || !f || u == f) return fail(MGC_EINVAL, "bad field pointers");
  if ((rc = validate_opts(g, o))) return rc;
  hipEvent_t e0, e1;
  HIPCHK(g, hipEventCreate(&e0));
  HIPCHK(g, hipEventCreate(&e1));
  HIPCHK(g, hipEventRecord(e0, g->stream));
  switch (o->outer) {
    case MGC_STATIONARY: rc = solve_stationary(g, u, f, o, st); break;
    case MGC_IR: rc = solve_ir(g, u, f, o, st); break;
    case MGC_BICGSTAB: rc = solve_bicgstab(g, u, f, o, st); break;
    default: rc = solve_fgmres(g, u, f, o, st); break;
  }
  if (rc == MGC_EHIP) return rc;
  mgc_status rc2 = MGC_OK;
  std::string keep = g_err;
  if (!hip_ok(g, hipEventRecord(e1, g->stream), "hipEventRecord") ||
      !hip_ok(g, hipEventSynchronize(e1), "hipEventSynchronize"))
    rc2 = MGC_EHIP;
  float ms = 0;
  (void)hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st) { st->t_solve_ms = ms; st->t_setup_ms = g->t_setup_ms; }
  if (rc2) return rc2;
  g_err = keep;
  if (!hip_ok(g, hipGetLastError(), "kernel launch")) return MGC_EHIP;
  return rc;
}

mgc_status mgc_solve_transpose(mgc_grid g, void* v, const void* gv, const mgc_solve_opts* o, mgc_stats* st) {
  mgc_status rc = check_ready(g);
  if (rc) return rc;
  if (!v || !gv || v == gv) return fail(MGC_EINVAL, "bad field pointers");
  if ((rc = validate_opts(g, o))) return rc;
  const int n = g->d.n, pitch = g->lv[0].pitch;
  const double2* w = g->at<const double2>(g->exact_w);
  double2* rhs = g->at<double2>(g->tt);                                // private to the transpose
  launch_weight(g->stream, n, pitch, w, 1, (const double2*)gv, rhs);   // W^{-1} g
  launch_weight(g->stream, n, pitch, w, 1, (const double2*)v, (double2*)v);   // y0 = W^{-1} v0
  rc = mgc_solve(g, v, rhs, o, st);
  if (rc == MGC_EHIP || rc == MGC_ESTATE || rc == MGC_EINVAL) return rc;
  launch_weight(g->stream, n, pitch, w, 0, (const double2*)v, (double2*)v);   // v = W y
  HIPCHK(g, hipGetLastError());
  HIPCHK(g, hipStreamSynchronize(g->stream));
  return rc;
}

mgc_status mgc_cross_section(mgc_grid g, const void* u, const void* chi, double k1, double k2,
                             double zeta[2], double* sigma) {
  mgc_status rc = check_ready(g);
  if (rc) return rc;
  if (g->d.gamma != 0.0) return fail(MGC_EINVAL, "the amplitudes are defined on a real interior (gamma = 0)");
  if (!u || !chi || !zeta || !(k1 > 0) || !(k2 > 0)) return fail(MGC_EINVAL, "bad arguments");
  const Axis& ax = g->exact;
  const int n = ax.n, j0 = ax.j0;
  std::vector<double> f1, f2, d1v, d2v;
  const std::vector<double>* tab = g->pot.kind == POT_TP ? nullptr : &g->v1r_host;
  test_function(ax, g->Z1, k1, f1, d1v, tab);
  test_function(ax, g->Z1, k2, f2, d2v, tab);
  std::vector<double> both(2 * (n + 1));
  for (int j = 0; j <= n; ++j) { both[j] = f1[j]; both[n + 1 + j] = f2[j]; }
  if ((rc = upload(g, g->zeta_f, both.data(), both.size() * sizeof(double)))) return rc;
  const double* d1 = g->at<const double>(g->zeta_f);
  double* part = g->at<double>(g->part);
  double* out = g->at<double>(g->scal);
  const double2* tm = nullptr;
  amp_source(g, g->stream, u, chi, tm);
  launch_zeta_part(g->stream, n, g->lv[0].pitch, j0, tm, d1, d1 + (n + 1), (const double2*)u,
                   (const double2*)chi, part);
  launch_sum_partials(g->stream, launch_vec_blocks(n), 2, part, out);
  HIPCHK(g, hipGetLastError());
  double hz[2];
  HIPCHK(g, hipMemcpyAsync(hz, out, sizeof(hz), hipMemcpyDeviceToHost, g->stream));
  HIPCHK(g, hipStreamSynchronize(g->stream));
  zeta[0] = hz[0];
  zeta[1] = hz[1];
  const double k0sq = k0sq_of(g);
  if (sigma) *sigma = 8.0 * M_PI * M_PI / k0sq * (hz[0] * hz[0] + hz[1] * hz[1]) / (k1 * k2);
  return MGC_OK;
}

mgc_status mgc_cross_section_sweep(mgc_grid g, const void* u, const void* chi, int npairs, const double* k1,
                                   const double* k2, double* zeta, double* sigma) {
  mgc_status rc = check_ready(g);
  if (rc) return rc;
  if (g->d.gamma != 0.0) return fail(MGC_EINVAL, "the amplitudes are defined on a real interior (gamma = 0)");
  if (!u || !chi || !k1 || !k2 || !zeta) return fail(MGC_EINVAL, "null argument");
  if (npairs < 1 || npairs > MGC_SWEEP_MAX) return fail(MGC_EINVAL, "npairs must lie in [1, MGC_SWEEP_MAX]");
  for (int a = 0; a < npairs; ++a)
    if (!(k1[a] > 0) || !(k2[a] > 0) || !std::isfinite(k1[a]) || !std::isfinite(k2[a]))
      return fail(MGC_EINVAL, "momenta must be finite and positive");
  const Axis& ax = g->exact;
  const int n = ax.n, top = std::min(ax.j0, n - 1);
  const int pp = (npairs + 63) / 64 * 64;
  // weighted test functions as [node][pair], zero for the padding pairs,
  // computed on the device from the momenta
  std::vector<double> kk(k1, k1 + npairs);
  kk.insert(kk.end(), k2, k2 + npairs);
  if ((rc = upload(g, g->sweep_k, kk.data(), kk.size() * sizeof(double)))) return rc;
  double* F = g->at<double>(g->sweep_f);
  launch_sweep_testfn(g->stream, n, ax.j0, ax.h, g->at<const double>(g->v1r), npairs, pp,
                      g->at<const double>(g->sweep_k), F);
  const double* F1T = F;
  double* out = g->at<double>(g->sweep_out);
  const double2* tm = nullptr;
  amp_source(g, g->stream, u, chi, tm);
  launch_zeta_sweep(g->stream, n, g->lv[0].pitch, top, pp, tm, F1T, F1T + (size_t)(n + 1) * pp,
                    (const double2*)u, (const double2*)chi, g->at<double>(g->sweep_part), out);
  HIPCHK(g, hipGetLastError());
  std::vector<double> hz((size_t)2 * pp);
  HIPCHK(g, hipMemcpyAsync(hz.data(), out, hz.size() * sizeof(double), hipMemcpyDeviceToHost, g->stream));
  HIPCHK(g, hipStreamSynchronize(g->stream));
  const double k0sq = k0sq_of(g);
  for (int a = 0; a < npairs; ++a) {
    zeta[2 * a] = hz[2 * a];
    zeta[2 * a + 1] = hz[2 * a + 1];
    if (sigma)
      sigma[a] = 8.0 * M_PI * M_PI / k0sq * (hz[2 * a] * hz[2 * a] + hz[2 * a + 1] * hz[2 * a + 1]) / (k1[a] * k2[a]);
  }
  return MGC_OK;
}

mgc_status mgc_cross_section_grad(mgc_grid g, const void* u, const void* chi, double k1, double k2,
                                  const mgc_solve_opts* opts, void* v, double dsigma[3], double zeta[2],
                                  double* sigma, mgc_stats* st) {
  mgc_status rc = check_ready(g);
  if (rc) return rc;
  if (g->pot.kind != POT_TP) return fail(MGC_EINVAL, "defined for the Temkin-Poet model only");
  if (g->d.gamma != 0.0) return fail(MGC_EINVAL, "the amplitudes are defined on a real interior (gamma = 0)");
  if (!u || !chi || !v || !dsigma || !(k1 > 0) || !(k2 > 0) || v == u || v == chi)
    return fail(MGC_EINVAL, "bad arguments");
  if (!(g->Z1 > 0)) return fail(MGC_EINVAL, "gradient needs Z1 > 0");
  if ((rc = validate_opts(g, opts))) return rc;
  const Axis& ax = g->exact;
  const int n = ax.n, j0 = ax.j0, pitch = g->lv[0].pitch;
  std::vector<double> f1, f2, d1, d2;
  test_function(ax, g->Z1, k1, f1, d1);
  test_function(ax, g->Z1, k2, f2, d2);
  std::vector<double> all(4 * (n + 1));
  for (int j = 0; j <= n; ++j) {
    all[j] = f1[j];
    all[(n + 1) + j] = f2[j];
    all[2 * (n + 1) + j] = d1[j];
    all[3 * (n + 1) + j] = d2[j];
  }
  if ((rc = upload(g, g->zeta_f, all.data(), all.size() * sizeof(double)))) return rc;
  const double* F = g->at<const double>(g->zeta_f);
  const double2* tm = exact_level(g).tm;
  double* part = g->at<double>(g->part);
  double* out = g->at<double>(g->scal);
  // zeta
  launch_zeta_part(g->stream, n, pitch, j0, tm, F, F + (n + 1), (const double2*)u, (const double2*)chi, part);
  launch_sum_partials(g->stream, launch_vec_blocks(n), 2, part, out);
  HIPCHK(g, hipGetLastError());
  double hz[2];
  HIPCHK(g, hipMemcpyAsync(hz, out, sizeof(hz), hipMemcpyDeviceToHost, g->stream));
  // adjoint: A^T v = d zeta / du
  launch_adj_rhs(g->stream, n, pitch, j0, tm, F, F + (n + 1), g->at<double2>(g->adj));
  HIPCHK(g, hipStreamSynchronize(g->stream));
  rc = mgc_solve_transpose(g, v, g->ws + g->adj, opts, st);
  if (rc != MGC_OK && rc != MGC_ENOCONV) return rc;
  const mgc_status solve_rc = rc;
  launch_sens_part(g->stream, n, pitch, j0, g->at<const double2>(g->exact_z), tm, F, F + (n + 1),
                   F + 2 * (n + 1), F + 3 * (n + 1), (const double2*)u, (const double2*)v,
                   (const double2*)chi, g->Z1, g->Z2, g->lam, g->E, part);
  launch_sum_partials(g->stream, launch_vec_blocks(n), 12, part, out);
  double s12[12];
  HIPCHK(g, hipMemcpyAsync(s12, out, sizeof(s12), hipMemcpyDeviceToHost, g->stream));
  HIPCHK(g, hipStreamSynchronize(g->stream));
  HIPCHK(g, hipGetLastError());
  const cd zt(hz[0], hz[1]);
  const double k0sq = 2.0 * g->E + g->Z1 * g->Z1;
  const double C = 8.0 * M_PI * M_PI / (k0sq * k1 * k2);
  const double sig = C * std::norm(zt);
  for (int q = 0; q < 3; ++q) {
    const cd dz(s12[2 * q] + s12[6 + 2 * q], s12[2 * q + 1] + s12[6 + 2 * q + 1]);
    dsigma[q] = 2.0 * C * std::real(std::conj(zt) * dz);
  }
  dsigma[0] += -sig * 2.0 * g->Z1 / k0sq;   // k0 depends on Z1
  if (zeta) { zeta[0] = hz[0]; zeta[1] = hz[1]; }
  if (sigma) *sigma = sig;
  return solve_rc;
}

}  // extern "C"

namespace {
// Gauss-Legendre rule on [-1, 1] (ascending nodes): the roots of P_N, found by
// Newton's method from x = cos(pi (i + 3/4) / (N + 1/2)), with P_N and P_N'
// from the three-term recurrence (j+1) P_{j+1} = (2j+1) x P_j - j P_{j-1};
// weights 2 / ((1 - x^2) P_N'(x)^2).
void gauss_legendre(int N, std::vector<double>& x, std::vector<double>& w) {
  x.assign(N, 0.0);
  w.assign(N, 0.0);
  for (int i = 0; i < N; ++i) {
    double r = std::cos(M_PI * (i + 0.75) / (N + 0.5)), dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = r;
      for (int j = 1; j < N; ++j) {
        const double p2 = ((2.0 * j + 1.0) * r * p1 - j * p0) / (j + 1.0);
        p0 = p1;
        p1 = p2;
      }
      if (N == 1) { p1 = r; p0 = 1.0; }
      dp = N * (r * p1 - p0) / (r * r - 1.0);
      const double dr = p1 / dp;
      r -= dr;
      if (std::abs(dr) < 1e-16) break;
    }
    x[N - 1 - i] = r;                        // ascending nodes
    w[N - 1 - i] = 2.0 / ((1.0 - r * r) * dp * dp);
  }
}

// Bound states of the exact x2 Hamiltonian -1/2 d2/dz2 - Z2/z (the
// one-body states phi_n of eq. single-ionization), held on the device for the
// single-ionisation sweep; recomputed after set_potential.
mgc_status ensure_si_states(mgc_grid g, int nstates) {
  if (g->si_count >= nstates) return MGC_OK;
  const Axis& ax = g->exact;
  std::vector<std::vector<cd>> phi;
  std::string err;
  if (!bound_states(ax, one_body(ax, g->pot, 2), nstates, 2, g->si_lam, phi, err)) return fail(MGC_ENUMERIC, err);
  std::vector<cd> tab((size_t)nstates * (ax.n + 1));
  for (int q = 0; q < nstates; ++q)
    for (int k = 0; k <= ax.n; ++k) tab[(size_t)q * (ax.n + 1) + k] = phi[q][k];
  mgc_status rc = upload_cplx<double>(g, g->si_tab, tab);
  if (rc) return rc;
  g->si_count = nstates;
  return MGC_OK;
}

// One amplitude sweep on stream st: weighted test functions (x1 side from
// kk[0 .. npairs), x2 side from kk[npairs .. 2 npairs) unless `bound` asks for
// the bound-state weights instead), the sweep over the field, and the copy of
// the 2 pp amplitude doubles into out.  kk and out are host buffers that must
// stay alive until st has synchronised.
mgc_status enqueue_sweep(mgc_grid g, const void* u, const void* chi, int npairs, const double* kk, int bound,
                         double* out, hipStream_t st) {
  const Axis& ax = g->exact;
  const int n = ax.n, top = std::min(ax.j0, n - 1);
  const int pp = (npairs + 63) / 64 * 64;
  double* F = g->at<double>(g->sweep_f);
  HIPCHK(g, hipMemcpyAsync(g->ws + g->sweep_k, kk, (size_t)2 * npairs * sizeof(double), hipMemcpyHostToDevice, st));
  launch_sweep_testfn(st, n, ax.j0, ax.h, g->at<const double>(g->v1r), npairs, pp, g->at<const double>(g->sweep_k),
                      F);
  if (bound > 0)
    launch_bound_weights(st, n, top, ax.j0, ax.h, bound, pp, g->at<const double2>(g->si_tab), F + (size_t)(n + 1) * pp);
  const double2* tm = nullptr;
  amp_source(g, st, u, chi, tm);
  launch_zeta_sweep(st, n, g->lv[0].pitch, top, pp, tm, F, F + (size_t)(n + 1) * pp,
                    (const double2*)u, (const double2*)chi, g->at<double>(g->sweep_part), g->at<double>(g->sweep_out));
  HIPCHK(g, hipGetLastError());
  HIPCHK(g, hipMemcpyAsync(out, g->ws + g->sweep_out, (size_t)2 * pp * sizeof(double), hipMemcpyDeviceToHost, st));
  return MGC_OK;
}

// Host staging of the cross sections of one handle.
struct XsecJob {
  int nstates = 0, nodes = 0;
  std::vector<double> kk_si, out_si, kk_dd, out_dd, wq, kn;
};

// Validate and build the momenta of both sweeps (nstates may be 0, nodes may
// be 0); enqueue them on st.
mgc_status enqueue_xsec(mgc_grid g, const void* u, const void* chi, int nstates, int nodes, XsecJob& J,
                        hipStream_t st) {
  if (g->d.gamma != 0.0) return fail(MGC_EINVAL, "the amplitudes are defined on a real interior (gamma = 0)");
  J.nstates = nstates;
  J.nodes = nodes;
  mgc_status rc;
  if (nstates > 0) {
    if ((rc = ensure_si_states(g, nstates))) return rc;
    J.kn.assign(nstates, 0.0);
    for (int q = 0; q < nstates; ++q) {
      const double e = g->E - g->si_lam[q].real();
      if (!(e > 0)) return fail(MGC_EINVAL, "single ionisation into state " + std::to_string(q + 1) +
                                                " is closed at this energy (E <= lambda_n)");
      J.kn[q] = std::sqrt(2.0 * e);
    }
    const int np = 2 * nstates;
    J.kk_si.assign((size_t)2 * np, 1.0);               // x2 side: replaced by the bound states
    for (int c = 0; c < np; ++c) J.kk_si[c] = J.kn[c / 2];
    J.out_si.assign((size_t)2 * ((np + 63) / 64 * 64), 0.0);
    if ((rc = enqueue_sweep(g, u, chi, np, J.kk_si.data(), nstates, J.out_si.data(), st))) return rc;
  }
  if (nodes > 0) {
    if (!(g->E > 0)) return fail(MGC_EINVAL, "double ionisation needs E > 0");
    std::vector<double> x, w;
    gauss_legendre(nodes, x, w);
    const double K = std::sqrt(2.0 * g->E);
    J.kk_dd.assign((size_t)2 * nodes, 0.0);
    J.wq.assign(nodes, 0.0);
    for (int q = 0; q < nodes; ++q) {
      const double a = (x[q] + 1.0) * M_PI / 4.0;
      J.kk_dd[q] = K * std::sin(a);
      J.kk_dd[nodes + q] = K * std::cos(a);
      J.wq[q] = w[q] * M_PI / 4.0;
    }
    J.out_dd.assign((size_t)2 * ((nodes + 63) / 64 * 64), 0.0);
    if ((rc = enqueue_sweep(g, u, chi, nodes, J.kk_dd.data(), 0, J.out_dd.data(), st))) return rc;
  }
  return MGC_OK;
}

// After the stream has synchronised: s_n from the pairs (2q: real part of
// the bound state, 2q+1: imaginary part) and sigma_tot from the rule.
void finish_xsec(mgc_grid g, const XsecJob& J, double* s, double* kn, double* sigma_tot, double* zeta) {
  for (int q = 0; q < J.nstates; ++q) {
    const double ar = J.out_si[4 * q], ai = J.out_si[4 * q + 1], br = J.out_si[4 * q + 2],
                 bi = J.out_si[4 * q + 3];
    if (s) {
      s[2 * q] = ar - bi;                      // (a) + i (b), a and b complex
      s[2 * q + 1] = ai + br;
    }
    if (kn) kn[q] = J.kn[q];
  }
  if (J.nodes > 0) {
    double acc = 0.0;
    for (int q = 0; q < J.nodes; ++q) {
      const double zr = J.out_dd[2 * q], zi = J.out_dd[2 * q + 1];
      acc += J.wq[q] * (zr * zr + zi * zi);
      if (zeta) {
        zeta[2 * q] = zr;
        zeta[2 * q + 1] = zi;
      }
    }
    const double k0sq = k0sq_of(g);
    if (sigma_tot) *sigma_tot = 8.0 * M_PI * M_PI / k0sq * acc;
  }
}
}  // namespace

extern "C" {

mgc_status mgc_single_ionization(mgc_grid g, const void* u, const void* chi, int nstates, double* s, double* kn) {
  mgc_status rc = check_ready(g);
  if (rc) return rc;
  if (!u || !chi || !s) return fail(MGC_EINVAL, "null argument");
  if (nstates < 1 || nstates > MGC_SI_MAX || nstates > g->d.n - 2)
    return fail(MGC_EINVAL, "nstates must lie in [1, MGC_SI_MAX] and below n - 1");
  XsecJob J;
  if ((rc = enqueue_xsec(g, u, chi, nstates, 0, J, g->stream))) return rc;
  HIPCHK(g, hipStreamSynchronize(g->stream));
  finish_xsec(g, J, s, kn, nullptr, nullptr);
  return MGC_OK;
}

mgc_status mgc_total_double_ionization(mgc_grid g, const void* u, const void* chi, int nodes, double* sigma_tot,
                                       double* zeta) {
  mgc_status rc = check_ready(g);
  if (rc) return rc;
  if (!u || !chi || !sigma_tot) return fail(MGC_EINVAL, "null argument");
  if (nodes < 1 || nodes > MGC_SWEEP_MAX) return fail(MGC_EINVAL, "nodes must lie in [1, MGC_SWEEP_MAX]");
  XsecJob J;
  if ((rc = enqueue_xsec(g, u, chi, 0, nodes, J, g->stream))) return rc;
  HIPCHK(g, hipStreamSynchronize(g->stream));
  finish_xsec(g, J, nullptr, nullptr, sigma_tot, zeta);
  return MGC_OK;
}

mgc_status mgc_set_kernel_timer(mgc_grid g, int kernel_class) {
  if (!g) return fail(MGC_EINVAL, "null handle");
  if (kernel_class < MGC_KT_NONE || kernel_class > MGC_KT_CCCS_EXPAND)
    return fail(MGC_EINVAL, "unknown kernel class");
  KernelTimer& t = g->kt;
  if (kernel_class != MGC_KT_NONE && !t.ev[0]) {
    for (int i = 0; i < 2 * KernelTimer::SLOTS; ++i) {
      HIPCHK(g, hipEventCreate(&t.ev[i]));
      HIPCHK(g, hipEventCreate(&t.fev[i]));
    }
  }
  t.which = kernel_class;
  t.used = 0;
  t.ms = 0;
  t.floor_ms = 0;
  t.total_bytes = 0;
  t.launches = 0;
  return MGC_OK;
}

mgc_status mgc_read_kernel_timer(mgc_grid g, mgc_kernel_timing* out) {
  if (!g || !out) return fail(MGC_EINVAL, "null argument");
  KernelTimer& t = g->kt;
  out->total_ms = t.ms;
  out->launches = t.launches;
  out->bytes = t.total_bytes;
  out->floor_ms = t.floor_ms;
  t.ms = 0;
  t.floor_ms = 0;
  t.total_bytes = 0;
  t.launches = 0;
  return MGC_OK;
}

}  // extern "C"

// ----------------------------------------------------------------------------
// Batched FGMRES: every solve's restart cycle is its own captured graph; the
// graphs of a round are launched over NSTREAMS streams so that they run
// concurrently, and the host synchronises once per round.
struct mgc_batch_s {
  static constexpr int NSTREAMS = 4;
  std::vector<mgc_grid> g;
  hipStream_t side[NSTREAMS] = {};         // default priority, non-blocking
  hipEvent_t start = nullptr;              // side streams wait for the batch stream
};

namespace {

struct BatchSolve {
  void* u = nullptr;
  const void* f = nullptr;
  double fn = 0, rel = 0;
  int it = 0, rs = 0, mm = 0;
  bool active = true;
  mgc_status status = MGC_OK;
  hipGraphExec_t exec = nullptr;           // restart cycle + true residual + report
  hipStream_t saved = nullptr;
};

// Capture solve s's restart cycle of mm steps, the true residual of the new
// iterate and the report (||r||^2, ||f||^2, steps used) into scal[REPORT..],
// and instantiate it.
mgc_status capture_cycle(mgc_grid g, BatchSolve& s, const mgc_solve_opts* o) {
  if (s.exec) {
    (void)hipGraphExecDestroy(s.exec);
    s.exec = nullptr;
  }
  HIPCHK(g, hipStreamBeginCapture(g->cap, hipStreamCaptureModeThreadLocal));
  enqueue_fgmres_cycle(g, s.u, o, o->tol * s.fn, s.mm, g->cap);
  enqueue_cycle_end(g, s.u, s.f, o->restart, g->cap);
  hipGraph_t graph = nullptr;
  HIPCHK(g, hipStreamEndCapture(g->cap, &graph));
  if (g->failed) {
    (void)hipGraphDestroy(graph);
    return MGC_EHIP;
  }
  hipError_t e = hipGraphInstantiate(&s.exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) s.exec = nullptr;
  HIPCHK(g, e);
  return MGC_OK;
}
}  // namespace

extern "C" {

mgc_status mgc_batch_create(const mgc_grid* grids, int count, mgc_batch* out) {
  if (!grids || !out || count < 1) return fail(MGC_EINVAL, "need grids, count >= 1 and an output handle");
  *out = nullptr;
  for (int i = 0; i < count; ++i) {
    if (!grids[i]) return fail(MGC_EINVAL, "null handle in batch");
    if (grids[i]->device != grids[0]->device) return fail(MGC_EINVAL, "batch handles must share one device");
    for (int j = 0; j < i; ++j)
      if (grids[j] == grids[i]) return fail(MGC_EINVAL, "a handle appears twice in the batch");
  }
  mgc_batch b = new mgc_batch_s;
  b->g.assign(grids, grids + count);
  for (int k = 0; k < mgc_batch_s::NSTREAMS; ++k)
    if (hipStreamCreateWithFlags(&b->side[k], hipStreamNonBlocking) != hipSuccess) {
      (void)mgc_batch_destroy(b);
      return fail(MGC_EHIP, "batch streams");
    }
  if (hipEventCreateWithFlags(&b->start, hipEventDisableTiming) != hipSuccess) {
    (void)mgc_batch_destroy(b);
    return fail(MGC_EHIP, "batch event");
  }
  *out = b;
  return MGC_OK;
}

mgc_status mgc_batch_solve(mgc_batch b, void* const* u, const void* const* f, const mgc_solve_opts* o,
                           mgc_stats* stats) {
  if (!b || !u || !f || !o) return fail(MGC_EINVAL, "null argument");
  if (o->outer != MGC_FGMRES) return fail(MGC_EINVAL, "batched solves run FGMRES");
  const int nb = (int)b->g.size();
  mgc_status rc;
  for (int i = 0; i < nb; ++i) {
    if ((rc = check_ready(b->g[i]))) return rc;
    if ((rc = validate_opts(b->g[i], o))) return rc;
    if (!u[i] || !f[i] || u[i] == f[i]) return fail(MGC_EINVAL, "bad field pointers in batch");
  }
  constexpr int NS = mgc_batch_s::NSTREAMS;
  mgc_grid g0 = b->g[0];
  hipStream_t s = g0->stream;
  std::vector<BatchSolve> v(nb);
  auto cleanup = [&]() {
    // an error may leave graphs of this round in flight: drain every stream
    // before their executable graphs are destroyed
    for (int k = 0; k < NS; ++k) (void)hipStreamSynchronize(b->side[k]);
    (void)hipStreamSynchronize(s);
    for (BatchSolve& x : v)
      if (x.exec) {
        (void)hipGraphExecDestroy(x.exec);
        x.exec = nullptr;
      }
    for (int i = 0; i < nb; ++i)
      if (v[i].saved) b->g[i]->stream = v[i].saved;
  };
  const auto t0 = std::chrono::steady_clock::now();
  // every handle works on the batch stream for the duration of the call
  for (int i = 0; i < nb; ++i) {
    v[i].saved = b->g[i]->stream;
    b->g[i]->stream = s;
    v[i].u = u[i];
    v[i].f = f[i];
  }
  // initial residuals W_0 = f - A u
  for (int i = 0; i < nb; ++i) {
    mgc_grid g = b->g[i];
    if (g->basis_dirty) {
      if (!hip_ok(g, hipMemsetAsync(g->at<double2>(g->W), 0,
                                    (size_t)(g->d.max_restart + 1) * g->field_bytes(0, P64), s),
                  "hipMemsetAsync")) {
        cleanup();
        return MGC_EHIP;
      }
      g->basis_dirty = false;
    }
    double rr = 0, ff = 0;
    if ((rc = exact_residual(g, u[i], f[i], g->at<double2>(g->W), &rr, &ff, gmres_state(g).nrm2))) {
      cleanup();
      return rc;
    }
    launch_gmres_begin(s, gmres_state(g), o->restart);
    v[i].fn = std::sqrt(ff);
    v[i].rel = std::sqrt(rr) / v[i].fn;
    if (stats) record(&stats[i], 0, v[i].rel);
    v[i].active = v[i].rel > o->tol && std::isfinite(v[i].rel);
  }
  if (!hip_ok(g0, hipEventRecord(b->start, s), "hipEventRecord")) {
    cleanup();
    return MGC_EHIP;
  }
  for (int k = 0; k < NS; ++k)
    if (!hip_ok(g0, hipStreamWaitEvent(b->side[k], b->start, 0), "hipStreamWaitEvent")) {
      cleanup();
      return MGC_EHIP;
    }
  const int m = o->restart;
  while (true) {
    int nact = 0;
    for (int i = 0; i < nb; ++i) {
      BatchSolve& x = v[i];
      if (!x.active) continue;
      const int mm = std::min(m, o->max_it - x.it);
      if (!x.exec || mm != x.mm) {
        x.mm = mm;
        if ((rc = capture_cycle(b->g[i], x, o))) {
          cleanup();
          return rc;
        }
      }
      if (!hip_ok(b->g[i], hipGraphLaunch(x.exec, b->side[nact % NS]), "hipGraphLaunch")) {
        cleanup();
        return MGC_EHIP;
      }
      ++nact;
    }
    if (nact == 0) break;
    for (int k = 0; k < std::min(NS, nact); ++k)
      if (!hip_ok(g0, hipStreamSynchronize(b->side[k]), "hipStreamSynchronize")) {
        cleanup();
        return MGC_EHIP;
      }
    for (int i = 0; i < nb; ++i) {
      BatchSolve& x = v[i];
      if (!x.active) continue;
      mgc_grid g = b->g[i];
      double r[3];
      if (!hip_ok(g, hipMemcpy(r, g->at<double>(g->scal) + REPORT, sizeof(r), hipMemcpyDeviceToHost),
                  "hipMemcpy")) {
        cleanup();
        return MGC_EHIP;
      }
      const int kused = (int)r[2];
      x.it += std::min(kused, x.mm);
      x.rel = std::sqrt(r[0]) / x.fn;
      ++x.rs;
      if (stats) record(&stats[i], x.rs, x.rel);
      if (x.rel <= o->tol || x.it >= o->max_it || !std::isfinite(x.rel)) x.active = false;
    }
  }
  const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  cleanup();
  mgc_status first = MGC_OK;
  for (int i = 0; i < nb; ++i) {
    BatchSolve& x = v[i];
    if (!std::isfinite(x.rel)) {
      x.status = MGC_ENUMERIC;
      b->g[i]->basis_dirty = true;
    } else if (x.rel > o->tol) {
      x.status = MGC_ENOCONV;
    }
    if (stats) {
      stats[i].iters = x.it;
      stats[i].vcycles = x.it;
      stats[i].relres = x.rel;
      stats[i].t_solve_ms = ms;
      stats[i].t_setup_ms = b->g[i]->t_setup_ms;
    }
    if (first == MGC_OK && x.status != MGC_OK) first = x.status;
  }
  if (first == MGC_ENUMERIC) return fail(MGC_ENUMERIC, "non-finite residual in a batched solve");
  if (first == MGC_ENOCONV) return fail(MGC_ENOCONV, "iteration limit reached in a batched solve");
  return MGC_OK;
}

mgc_status mgc_batch_cross_sections(mgc_batch b, const void* const* u, const void* const* chi, int nodes,
                                    int nstates, double* sigma_tot, double* s) {
  if (!b || !u || !chi) return fail(MGC_EINVAL, "null argument");
  if (nodes < 0 || nodes > MGC_SWEEP_MAX || nstates < 0 || nstates > MGC_SI_MAX || (nodes == 0 && nstates == 0))
    return fail(MGC_EINVAL, "need 0 <= nodes <= MGC_SWEEP_MAX, 0 <= nstates <= MGC_SI_MAX, not both zero");
  if ((nodes > 0 && !sigma_tot) || (nstates > 0 && !s)) return fail(MGC_EINVAL, "null output array");
  const int nb = (int)b->g.size();
  mgc_status rc;
  for (int i = 0; i < nb; ++i) {
    if ((rc = check_ready(b->g[i]))) return rc;
    if (!u[i] || !chi[i]) return fail(MGC_EINVAL, "null field pointer in batch");
    if (nstates > b->g[i]->d.n - 2) return fail(MGC_EINVAL, "nstates must lie below n - 1 on every grid");
    if (nodes > 0 && !(b->g[i]->E > 0)) return fail(MGC_EINVAL, "double ionisation needs E > 0 on every grid");
  }
  constexpr int NS = mgc_batch_s::NSTREAMS;
  mgc_grid g0 = b->g[0];
  // the side streams start after the work already on the handles' streams
  for (int i = 0; i < nb; ++i) {
    if (!hip_ok(g0, hipEventRecord(b->start, b->g[i]->stream), "hipEventRecord")) return MGC_EHIP;
    for (int k = 0; k < NS; ++k)
      if (!hip_ok(g0, hipStreamWaitEvent(b->side[k], b->start, 0), "hipStreamWaitEvent")) return MGC_EHIP;
  }
  std::vector<XsecJob> jobs(nb);
  for (int i = 0; i < nb; ++i) {
    rc = enqueue_xsec(b->g[i], u[i], chi[i], nstates, nodes, jobs[i], b->side[i % NS]);
    if (rc) {
      for (int k = 0; k < NS; ++k) (void)hipStreamSynchronize(b->side[k]);
      return rc;
    }
  }
  for (int k = 0; k < NS; ++k)
    if (!hip_ok(g0, hipStreamSynchronize(b->side[k]), "hipStreamSynchronize")) return MGC_EHIP;
  for (int i = 0; i < nb; ++i)
    finish_xsec(b->g[i], jobs[i], nstates > 0 ? s + (size_t)2 * nstates * i : nullptr, nullptr,
                nodes > 0 ? sigma_tot + i : nullptr, nullptr);
  return MGC_OK;
}

mgc_status mgc_batch_destroy(mgc_batch b) {
  if (!b) return fail(MGC_EINVAL, "null batch");
  for (hipStream_t& st : b->side)
    if (st) (void)hipStreamDestroy(st);
  if (b->start) (void)hipEventDestroy(b->start);
  delete b;
  return MGC_OK;
}

mgc_status mgc_destroy_grid(mgc_grid g) {
  if (!g) return fail(MGC_EINVAL, "null handle");
  if (g->graph.exec) (void)hipGraphExecDestroy(g->graph.exec);
  if (g->plain.exec) (void)hipGraphExecDestroy(g->plain.exec);
  if (g->bicg_graph.exec) (void)hipGraphExecDestroy(g->bicg_graph.exec);
  for (hipEvent_t e : g->kt.ev)
    if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : g->kt.fev)
    if (e) (void)hipEventDestroy(e);
  if (g->cap) (void)hipStreamDestroy(g->cap);
  delete g;
  return MGC_OK;
}

}  // extern "C"
