// Host-side run of the batched-solve bookkeeping of the MG-CCCS library under
// AddressSanitizer, with the HIP runtime and the kernels replaced by
// stub_hip.cpp (no GPU needed).  It builds the handles of a batch workload
// (one line per solve: n L E M levels), runs mgc_batch_solve over several
// restart rounds in which the solves finish at different rounds, runs each
// solve alone with mgc_solve, runs the batch again with an iteration limit
// between the solves' needs, takes the cross sections of every energy in one
// batched call, and destroys everything.  Exit status 0 and no
// sanitizer report mean the host code touched only memory it owned.
#include <sys/mman.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../../include/mgcccs.h"

extern "C" void stub_reset_iterates();   // stub_hip.cpp

namespace {
// "device" buffer: anonymous pages followed by one inaccessible page, so that
// a write past the end faults at once
struct Buf {
  void* p = nullptr;
  size_t bytes = 0, mapped = 0;
};
Buf dev_alloc(size_t bytes) {
  const size_t page = 4096;
  Buf b;
  b.bytes = bytes;
  b.mapped = (bytes + page - 1) / page * page + page;
  char* base = (char*)mmap(nullptr, b.mapped, PROT_READ | PROT_WRITE, MAP_PRIVATE | MAP_ANONYMOUS | MAP_NORESERVE,
                           -1, 0);
  if (base == MAP_FAILED) {
    std::perror("mmap");
    std::exit(3);
  }
  mprotect(base + b.mapped - page, page, PROT_NONE);
  // the library wants 256-byte alignment; the end of the usable range sits
  // right before the guard page
  b.p = base + (b.mapped - page - (bytes + 255) / 256 * 256);
  return b;
}
void dev_free(Buf& b) {
  const size_t page = 4096;
  char* base = (char*)b.p - (b.mapped - page - (b.bytes + 255) / 256 * 256);
  munmap(base, b.mapped);
  b.p = nullptr;
}
#define CHECK(x)                                                                 \
  do {                                                                           \
    mgc_status rc_ = (x);                                                        \
    if (rc_ != MGC_OK) {                                                         \
      std::fprintf(stderr, "%s -> %d (%s)\n", #x, (int)rc_, mgc_last_error());   \
      return 1;                                                                  \
    }                                                                            \
  } while (0)
}  // namespace

int main(int argc, char** argv) {
  if (argc < 2) {
    std::fprintf(stderr, "usage: %s workload.txt\n", argv[0]);
    return 2;
  }
  FILE* fh = std::fopen(argv[1], "r");
  if (!fh) return 2;
  struct W { int n, M, levels; double L, E; };
  std::vector<W> wl;
  W w;
  while (std::fscanf(fh, "%d %lf %lf %d %d", &w.n, &w.L, &w.E, &w.M, &w.levels) == 5) wl.push_back(w);
  std::fclose(fh);
  const int nb = (int)wl.size();
  std::vector<mgc_grid> g(nb);
  std::vector<Buf> ws(nb), ub(nb), fb(nb);
  std::vector<void*> up(nb);
  std::vector<const void*> fp(nb);
  for (int i = 0; i < nb; ++i) {
    mgc_grid_desc d{};
    d.n = wl[i].n;
    d.L = wl[i].L;
    d.R0 = 0.75 * wl[i].L;
    d.theta = M_PI / 6;
    d.levels = wl[i].levels;
    d.M = d.Lch = wl[i].M;
    d.omega = 2.0 / 3.0;
    d.nu1 = d.nu2 = 1;
    d.pc_gamma = 15.0 * M_PI / 180.0;
    d.pc_first_level = 1;
    d.max_restart = 10;
    d.precisions = 3;
    CHECK(mgc_create_grid(&d, nullptr, &g[i]));
    size_t bytes = 0;
    CHECK(mgc_workspace_bytes(g[i], &bytes));
    ws[i] = dev_alloc(bytes);
    CHECK(mgc_bind_workspace(g[i], ws[i].p, bytes));
    CHECK(mgc_set_potential(g[i], 1.0, 1.0, 1.0));
    CHECK(mgc_set_energy(g[i], wl[i].E));
    int pitch = 0;
    CHECK(mgc_field_pitch(g[i], 0, &pitch));
    const size_t fbytes = (size_t)(wl[i].n + 1) * pitch * 16;
    ub[i] = dev_alloc(fbytes);
    fb[i] = dev_alloc(fbytes);
    up[i] = ub[i].p;
    fp[i] = fb[i].p;
  }
  std::printf("%d handles set up\n", nb);
  mgc_batch b = nullptr;
  CHECK(mgc_batch_create(g.data(), nb, &b));
  mgc_solve_opts o{};
  o.outer = MGC_FGMRES;
  o.inner = MGC_FP32;
  o.restart = 10;
  o.max_it = 20000;
  o.inner_cycles = 1;
  o.tol = 1e-10;
  std::vector<std::vector<double>> hist(nb, std::vector<double>(64));
  std::vector<mgc_stats> st(nb);
  for (int i = 0; i < nb; ++i) {
    st[i] = mgc_stats{};
    st[i].hist = hist[i].data();
    st[i].hist_cap = 64;
  }
  CHECK(mgc_batch_solve(b, up.data(), fp.data(), &o, st.data()));
  int rounds_min = 1 << 30, rounds_max = 0;
  for (int i = 0; i < nb; ++i) {
    if (!(st[i].relres <= o.tol)) {
      std::fprintf(stderr, "solve %d did not converge: %g\n", i, st[i].relres);
      return 1;
    }
    rounds_min = std::min(rounds_min, st[i].hist_len - 1);
    rounds_max = std::max(rounds_max, st[i].hist_len - 1);
  }
  std::printf("batch: restart rounds per solve %d .. %d\n", rounds_min, rounds_max);
  // each solve alone, FP64 and FP32 cycles
  stub_reset_iterates();
  for (int i = 0; i < nb; ++i) {
    mgc_stats s1{};
    o.inner = (i % 2) ? MGC_FP32 : MGC_FP64;
    CHECK(mgc_solve(g[i], up[i], fp[i], &o, &s1));
    if (s1.iters != st[i].iters) {
      std::fprintf(stderr, "solve %d: %d iterations alone, %d in the batch\n", i, s1.iters, st[i].iters);
      return 1;
    }
  }
  // an iteration limit between the solves' needs: some stop early
  o.inner = MGC_FP32;
  o.max_it = (rounds_min + rounds_max) / 2 * o.restart + 3;
  stub_reset_iterates();
  mgc_status rc = mgc_batch_solve(b, up.data(), fp.data(), &o, st.data());
  if (rc != MGC_ENOCONV) {
    std::fprintf(stderr, "limited batch returned %d\n", (int)rc);
    return 1;
  }
  int stopped = 0;
  for (int i = 0; i < nb; ++i) stopped += st[i].relres > o.tol;
  std::printf("limited batch: %d of %d stopped at the limit\n", stopped, nb);
  // cross sections of every energy of the batch in one call
  std::vector<double> sig(nb), sn((size_t)nb * 2 * 2);
  CHECK(mgc_batch_cross_sections(b, up.data(), fp.data(), 24, 2, sig.data(), sn.data()));
  std::printf("batch cross sections done\n");
  CHECK(mgc_batch_destroy(b));
  for (int i = 0; i < nb; ++i) {
    CHECK(mgc_destroy_grid(g[i]));
    dev_free(ws[i]);
    dev_free(ub[i]);
    dev_free(fb[i]);
  }
  std::printf("OK\n");
  return 0;
}
