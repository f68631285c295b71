// Host-only stand-in for the HIP runtime and the kernel launchers of the
// MG-CCCS library, so that the library's host code (api.cpp, setup.cpp) can be
// built with AddressSanitizer and run on a machine without a GPU.
//
// "Device memory" is ordinary host memory.  Streams run their work at once,
// except while a stream is being captured: then each operation is appended to
// the capture, and a launched executable graph runs the captured operations in
// order.  Kernels do nothing, except the few whose results steer the host:
//   * a residual pass with a reduction target (the true residual of a solve)
//     writes ||r||^2 and ||f||^2 = 1, where ||r||^2 starts at 1 for every
//     iterate and each FGMRES update of the iterate shrinks it by a factor
//     that depends on the grid size, so that solves of different sizes need
//     different numbers of restart rounds;
//   * the FGMRES least-squares step reports the steps used (mm);
//   * the batch report copies ||r||^2, ||f||^2 and the steps used.
// Graph objects, executable graphs, streams and events are heap objects, so
// AddressSanitizer sees every use after free and every leak of them.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <functional>
#include <map>
#include <vector>

#include "../../paper_1412_1953_amd/csrc/launch.h"

namespace {
using Op = std::function<void()>;
struct FakeStream {
  std::vector<Op>* cap = nullptr;          // active capture, or null
};
struct FakeGraph {
  std::vector<Op> ops;
};
struct FakeExec {
  std::vector<Op> ops;
};
struct FakeEvent {
  int recorded = 0;
};
FakeStream g_null_stream;
hipError_t g_last = hipSuccess;

FakeStream* fs(hipStream_t s) { return s ? reinterpret_cast<FakeStream*>(s) : &g_null_stream; }
void enqueue(hipStream_t s, Op op) {
  FakeStream* f = fs(s);
  if (f->cap) f->cap->push_back(std::move(op));
  else op();
}
// ||f - A u||^2 of each iterate u (keyed by its device address), 1 until the
// first update; every FGMRES update of u shrinks it by a factor that depends
// on the grid size
std::map<const void*, double> g_res;
double shrink(int n) { return n <= 64 ? 0.05 : n <= 128 ? 0.1 : n <= 256 ? 0.15 : n <= 512 ? 0.25 : 0.4; }
}  // namespace

// Between phases of the harness: every iterate starts again at residual 1.
extern "C" void stub_reset_iterates() { g_res.clear(); }

extern "C" {
hipError_t hipGetLastError(void) {
  hipError_t e = g_last;
  g_last = hipSuccess;
  return e;
}
const char* hipGetErrorString(hipError_t) { return "stub error"; }
hipError_t hipGetDevice(int* d) {
  *d = 0;
  return hipSuccess;
}
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned int) {
  *s = reinterpret_cast<hipStream_t>(new FakeStream);
  return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
  delete reinterpret_cast<FakeStream*>(s);
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t s) {
  return fs(s)->cap ? hipErrorStreamCaptureUnsupported : hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t e, unsigned int) {
  if (!e) return hipErrorInvalidValue;
  return hipSuccess;
}
hipError_t hipEventCreate(hipEvent_t* e) {
  *e = reinterpret_cast<hipEvent_t>(new FakeEvent);
  return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { return hipEventCreate(e); }
hipError_t hipEventDestroy(hipEvent_t e) {
  delete reinterpret_cast<FakeEvent*>(e);
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
  FakeEvent* ev = reinterpret_cast<FakeEvent*>(e);
  enqueue(s, [ev] { ev->recorded++; });
  return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t e) { return e ? hipSuccess : hipErrorInvalidValue; }
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b) {
  *ms = (reinterpret_cast<FakeEvent*>(a)->recorded && reinterpret_cast<FakeEvent*>(b)->recorded) ? 0.001f : 0.0f;
  return hipSuccess;
}
hipError_t hipMemcpy(void* dst, const void* src, size_t bytes, hipMemcpyKind) {
  std::memcpy(dst, src, bytes);
  return hipSuccess;
}
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind, hipStream_t s) {
  enqueue(s, [=] { std::memcpy(dst, src, bytes); });
  return hipSuccess;
}
hipError_t hipMemsetAsync(void* dst, int v, size_t bytes, hipStream_t s) {
  enqueue(s, [=] { std::memset(dst, v, bytes); });
  return hipSuccess;
}
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) {
  FakeStream* f = fs(s);
  if (f->cap) return hipErrorIllegalState;
  f->cap = new std::vector<Op>;
  return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g) {
  FakeStream* f = fs(s);
  if (!f->cap) return hipErrorIllegalState;
  FakeGraph* gr = new FakeGraph;
  gr->ops = std::move(*f->cap);
  delete f->cap;
  f->cap = nullptr;
  *g = reinterpret_cast<hipGraph_t>(gr);
  return hipSuccess;
}
hipError_t hipStreamIsCapturing(hipStream_t s, hipStreamCaptureStatus* st) {
  *st = fs(s)->cap ? hipStreamCaptureStatusActive : hipStreamCaptureStatusNone;
  return hipSuccess;
}
hipError_t hipStreamGetCaptureInfo_v2(hipStream_t s, hipStreamCaptureStatus* st, unsigned long long* id,
                                      hipGraph_t* g, const hipGraphNode_t** deps, size_t* nd) {
  *st = fs(s)->cap ? hipStreamCaptureStatusActive : hipStreamCaptureStatusNone;
  if (id) *id = 0;
  if (g) *g = nullptr;
  if (deps) *deps = nullptr;
  if (nd) *nd = 0;
  return hipSuccess;
}
hipError_t hipGraphAddEventRecordNode(hipGraphNode_t* node, hipGraph_t, const hipGraphNode_t*, size_t,
                                      hipEvent_t) {
  *node = nullptr;
  return hipSuccess;
}
hipError_t hipStreamUpdateCaptureDependencies(hipStream_t, hipGraphNode_t*, size_t, unsigned int) {
  return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t* x, hipGraph_t g, hipGraphNode_t*, char*, size_t) {
  FakeExec* e = new FakeExec;
  e->ops = reinterpret_cast<FakeGraph*>(g)->ops;
  *x = reinterpret_cast<hipGraphExec_t>(e);
  return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g) {
  delete reinterpret_cast<FakeGraph*>(g);
  return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t x) {
  delete reinterpret_cast<FakeExec*>(x);
  return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t x, hipStream_t s) {
  FakeExec* e = reinterpret_cast<FakeExec*>(x);
  if (fs(s)->cap) return hipErrorIllegalState;
  for (Op& op : e->ops) op();
  return hipSuccess;
}
}  // extern "C"

namespace mgc {

// block counts of the reductions: stand-ins (they size scratch regions of the
// workspace layout, which the stub kernels never read)
int launch_stencil_blocks(int n) { return (n - 1 + 63) / 64; }
int launch_vec_blocks(int n) { return (n - 1 + 63) / 64; }
int launch_cccs_reduce_blocks(int n) { return (n - 1 + 31) / 32; }
int zeta_sweep_blocks(int top) { return (top + 7) / 8; }

template <typename T, typename TU, typename TF, typename TO>
void launch_stencil(hipStream_t s, const Level<T>&, const void* u, const void*, void*, int, double* part,
                    Finish fin) {
  if (!fin.out) {
    // partials only: the model keeps the two sums in part[0..1]
    enqueue(s, [part, u] {
      if (!part) return;
      auto it = g_res.find(u);
      part[0] = it == g_res.end() ? 1.0 : it->second;
      part[1] = 1.0;
    });
    return;
  }
  enqueue(s, [fin, u] {
    auto it = g_res.find(u);
    const double r2 = it == g_res.end() ? 1.0 : it->second;
    fin.out[0] = r2;
    fin.out[1] = 1.0;
    if (fin.copy_to) fin.copy_to[0] = r2;
  });
}
template void launch_stencil<double, double, double, double>(hipStream_t, const Level<double>&, const void*,
                                                             const void*, void*, int, double*, Finish);
template void launch_stencil<float, float, float, float>(hipStream_t, const Level<float>&, const void*,
                                                         const void*, void*, int, double*, Finish);

#define MGC_NOP(s) enqueue((s), [] {})
template <typename T>
void launch_jacobi(hipStream_t s, const Level<T>&, const void*, const void*, void*, double) { MGC_NOP(s); }
template <typename T>
void launch_resid_restrict(hipStream_t s, const Level<T>&, const void*, const void*, void*, int) { MGC_NOP(s); }
template <typename T>
void launch_prolong_add(hipStream_t s, int, int, void*, const void*, int) { MGC_NOP(s); }
template <typename T>
void launch_coarse_solve(hipStream_t s, const double2*, int, int, const void*, void*) { MGC_NOP(s); }
template <typename T>
void launch_s1_zero(hipStream_t s, const Level<T>&, const void*, const double*, double, void*, int, bool) {
  MGC_NOP(s);
}
template <typename T>
void launch_s2_zero(hipStream_t s, const Level<T>&, const void*, const double*, double, const void*, int, void*,
                    bool) {
  MGC_NOP(s);
}
template <typename T>
void launch_s1_pair(hipStream_t s, const Level<T>&, const Level<T>&, const void*, const double*, double, void*, int,
                    void*, int) {
  MGC_NOP(s);
}
template <typename T>
void launch_s2_pair(hipStream_t s, const Level<T>&, const Level<T>&, const void*, const double*, double,
                    const void*, const void*, int, void*) {
  MGC_NOP(s);
}
template <typename T>
void launch_tail(hipStream_t s, const TailArgs<T>&, bool) { MGC_NOP(s); }
template <typename T>
void launch_cccs(hipStream_t s, const Level<T>&, void*, const void*, const double*, const ChanTab<T>&,
                 const ChanSys<T>&, const ChanSys<T>&, const CccsScratch&, const MarkHook* hook) {
  for (int kind = 1; kind <= 3; ++kind) {
    if (hook && hook->fn && hook->kind == kind) hook->fn(hook->ctx, s, 0);
    MGC_NOP(s);
    if (hook && hook->fn && hook->kind == kind) hook->fn(hook->ctx, s, 1);
  }
}
#define MGC_STUB_INST(T)                                                                                      \
  template void launch_jacobi<T>(hipStream_t, const Level<T>&, const void*, const void*, void*, double);      \
  template void launch_resid_restrict<T>(hipStream_t, const Level<T>&, const void*, const void*, void*, int); \
  template void launch_prolong_add<T>(hipStream_t, int, int, void*, const void*, int);                        \
  template void launch_coarse_solve<T>(hipStream_t, const double2*, int, int, const void*, void*);           \
  template void launch_s1_zero<T>(hipStream_t, const Level<T>&, const void*, const double*, double, void*, int, \
                                  bool);                                                                      \
  template void launch_s2_zero<T>(hipStream_t, const Level<T>&, const void*, const double*, double, const void*, \
                                  int, void*, bool);                                                          \
  template void launch_s1_pair<T>(hipStream_t, const Level<T>&, const Level<T>&, const void*, const double*,   \
                                  double, void*, int, void*, int);                                            \
  template void launch_s2_pair<T>(hipStream_t, const Level<T>&, const Level<T>&, const void*, const double*,   \
                                  double, const void*, const void*, int, void*);                              \
  template void launch_tail<T>(hipStream_t, const TailArgs<T>&, bool);                                        \
  template void launch_cccs<T>(hipStream_t, const Level<T>&, void*, const void*, const double*,               \
                               const ChanTab<T>&, const ChanSys<T>&, const ChanSys<T>&, const CccsScratch&,   \
                               const MarkHook*);
MGC_STUB_INST(double)
MGC_STUB_INST(float)

template <typename TZ>
void launch_apply_dot(hipStream_t s, const Level<double>&, const void*, size_t, const double2*, int, double2*,
                      double*) {
  MGC_NOP(s);
}
template void launch_apply_dot<double>(hipStream_t, const Level<double>&, const void*, size_t, const double2*, int,
                                       double2*, double*);
template void launch_apply_dot<float>(hipStream_t, const Level<double>&, const void*, size_t, const double2*, int,
                                      double2*, double*);
void launch_axpy_pass(hipStream_t s, int, int, size_t, const double2*, int, double2*, float2*, const double*,
                      double*, const GmresState&) {
  MGC_NOP(s);
}
void launch_reorth_step(hipStream_t s, int, int, size_t, const double2*, int J, double2*, float2*, const double*,
                        const double*, double*, const GmresState& st, int, int mm, double, double) {
  int* k = st.kused;
  if (J == mm) enqueue(s, [k, mm] { k[0] = mm; });   // the cycle's least squares
  else MGC_NOP(s);
}
template <typename TZ>
void launch_update(hipStream_t s, int n, int, size_t, const void*, int, const double2*, double2* u) {
  const double q = shrink(n);
  enqueue(s, [u, q] {
    auto it = g_res.find(u);
    g_res[u] = (it == g_res.end() ? 1.0 : it->second) * q * q;
  });
}
template void launch_update<double>(hipStream_t, int, int, size_t, const void*, int, const double2*, double2*);
template void launch_update<float>(hipStream_t, int, int, size_t, const void*, int, const double2*, double2*);
template <typename TI, typename TO>
void launch_scale_copy(hipStream_t s, int, int, int, const void*, const double*, void*) { MGC_NOP(s); }
template void launch_scale_copy<double, double>(hipStream_t, int, int, int, const void*, const double*, void*);
template void launch_scale_copy<double, float>(hipStream_t, int, int, int, const void*, const double*, void*);
template void launch_scale_copy<float, double>(hipStream_t, int, int, int, const void*, const double*, void*);
template void launch_scale_copy<float, float>(hipStream_t, int, int, int, const void*, const double*, void*);
void launch_weight(hipStream_t s, int, int, const double2*, int, const double2*, double2*) { MGC_NOP(s); }
void launch_sum_partials(hipStream_t s, int, int nq, const double*, double* out) {
  enqueue(s, [=] {
    for (int q = 0; q < nq; ++q) out[q] = 0.0;
  });
}
void launch_gmres_begin(hipStream_t s, const GmresState&, int) { MGC_NOP(s); }
void launch_ir_scale(hipStream_t s, const double*, double, double* sc) {
  enqueue(s, [sc] {
    sc[0] = 1.0;
    sc[2] = 1.0;
    sc[3] = 0.0;
  });
}
void launch_copy_scalar(hipStream_t s, const double* src, double* dst) {
  enqueue(s, [=] { dst[0] = src[0]; });
}
void launch_cycle_end(hipStream_t s, int, const double* part, double* scal, const GmresState& st, int,
                      double* rep) {
  double* nrm2 = st.nrm2;
  const int* kused = st.kused;
  enqueue(s, [=] {
    scal[0] = part[0];
    scal[1] = part[1];
    nrm2[0] = part[0];
    rep[0] = scal[0];
    rep[1] = scal[1];
    rep[2] = (double)kused[0];
  });
}
void launch_fill_zero(hipStream_t s, void* p, size_t bytes) {
  enqueue(s, [=] { std::memset(p, 0, bytes); });
}
void launch_rhs_tp(hipStream_t s, int, int, int, const double2*, double, double, double, double, double2*) {
  MGC_NOP(s);
}
void launch_adj_rhs(hipStream_t s, int, int, int, const double2*, const double*, const double*, double2*) {
  MGC_NOP(s);
}
void launch_sens_part(hipStream_t s, int, int, int, const double2*, const double2*, const double*, const double*,
                      const double*, const double*, const double2*, const double2*, const double2*, double, double,
                      double, double, double*) {
  MGC_NOP(s);
}
void launch_zeta_part(hipStream_t s, int, int, int, const double2*, const double*, const double*, const double2*,
                      const double2*, double*) {
  MGC_NOP(s);
}
void launch_sweep_testfn(hipStream_t s, int, int, double, const double*, int, int, const double*, double*) { MGC_NOP(s); }
void launch_src_v12(hipStream_t s, int, int, const double2*, const double2*, const double2*, double2*) { MGC_NOP(s); }
void launch_bound_weights(hipStream_t s, int, int, int, double, int, int, const double2*, double*) { MGC_NOP(s); }
void launch_bicg_init(hipStream_t s, double*, const double*) { MGC_NOP(s); }
template <typename T>
void launch_gmres3_smooth(hipStream_t s, const Level<T>&, void*, const void*, void*, size_t, double*, double*) {
  MGC_NOP(s);
}
template void launch_gmres3_smooth<double>(hipStream_t, const Level<double>&, void*, const void*, void*, size_t,
                                           double*, double*);
template void launch_gmres3_smooth<float>(hipStream_t, const Level<float>&, void*, const void*, void*, size_t, double*,
                                          double*);
int gmres3_part_doubles(int n) { return 8 * n; }
template <typename T>
void launch_add(hipStream_t s, int, int, const void*, void*) { MGC_NOP(s); }
template <typename T>
void launch_gs_tail(hipStream_t s, const GsTailArgs<T>&) { MGC_NOP(s); }
template void launch_gs_tail<double>(hipStream_t, const GsTailArgs<double>&);
template void launch_gs_tail<float>(hipStream_t, const GsTailArgs<float>&);
template void launch_add<double>(hipStream_t, int, int, const void*, void*);
template void launch_add<float>(hipStream_t, int, int, const void*, void*);
void launch_bicg_p(hipStream_t s, int, int, const double2*, const double2*, double2*, float2*, const double*) {
  MGC_NOP(s);
}
void launch_bicg_s(hipStream_t s, int, int, const double*, double*, const double2*, const double2*, double2*, float2*,
                   double*) {
  MGC_NOP(s);
}
template <typename TZ>
void launch_bicg_x(hipStream_t s, int, int, const double*, const double*, double, double*, const void*, const void*,
                   const double2*, const double2*, const double2*, double2*, double2*, double*) {
  MGC_NOP(s);
}
template void launch_bicg_x<double>(hipStream_t, int, int, const double*, const double*, double, double*, const void*,
                                    const void*, const double2*, const double2*, const double2*, double2*, double2*,
                                    double*);
template void launch_bicg_x<float>(hipStream_t, int, int, const double*, const double*, double, double*, const void*,
                                   const void*, const double2*, const double2*, const double2*, double2*, double2*,
                                   double*);
void launch_bicg_rho(hipStream_t s, int, const double*, double*, double*) { MGC_NOP(s); }
void launch_zeta_sweep(hipStream_t s, int, int, int, int, const double2*, const double*, const double*,
                       const double2*, const double2*, double*, double* out) {
  MGC_NOP(s);
  (void)out;
}

}  // namespace mgc
