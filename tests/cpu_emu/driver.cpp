// Runs the engine's host code through the C ABI on the CPU device emulation
// (kernels_emu.cpp), in the pattern of the batched sweeps: several contexts
// advanced in lockstep by sadmrg_batch_sweep, whose per-problem preparation
// and update run on the library's host worker threads, in FP64 and in mixed
// precision, with checkpointed blocks, followed by separate sweeps and the
// energy adjoint, and (unless --no-inject is given) injected device failures
// (in the worker threads, beside the planning thread, in shared and single
// sigma launches) that must come back as errors; then (unless --no-block is
// given) the block-Jacobi decomposition of a larger problem's wide sectors
// against the one-workgroup decomposition.  Built with -fsanitize=thread or -fsanitize=address by
// tests/test_cpu_emulation.py; prints one summary line and returns nonzero on
// an error or an inconsistent result.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/sadmrg.h"

namespace sadmrg {  // switches of the emulated device layer (kernels_emu.cpp)
extern std::atomic<long> emu_svd_block_pairs_run;
extern std::atomic<bool> emu_svd_block_off;
extern std::atomic<int> emu_fail_gathers;
extern std::atomic<int> emu_fail_gemms;
}  // namespace sadmrg

namespace {

uint64_t mix(uint64_t x) {  // SplitMix64 finaliser
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}
double gauss(uint64_t& s) {  // Box-Muller on two counter draws
  const double u1 = ((mix(++s) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
  const double u2 = ((mix(++s) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
  return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
}

// h_ii = -2 + 3i/(L-1), small symmetric off-diagonal h; (ij|kl) = sum_P B_ij B_kl
void integrals(int L, uint64_t seed, std::vector<double>& h, std::vector<double>& eri) {
  uint64_t s = seed * 1000003ull;
  h.assign((size_t)L * L, 0.0);
  for (int i = 0; i < L; ++i) {
    h[(size_t)i * L + i] = -2.0 + 3.0 * i / (L - 1);
    for (int j = 0; j < i; ++j) h[(size_t)i * L + j] = h[(size_t)j * L + i] = 0.02 * gauss(s);
  }
  eri.assign((size_t)L * L * L * L, 0.0);
  std::vector<double> B((size_t)L * L);
  for (int P = 0; P < 2 * L; ++P) {
    for (int i = 0; i < L; ++i)
      for (int j = 0; j <= i; ++j) B[(size_t)i * L + j] = B[(size_t)j * L + i] = 0.3 / std::sqrt(1.0 + i - j) * gauss(s);
    for (size_t a = 0; a < (size_t)L * L; ++a)
      for (size_t b = 0; b < (size_t)L * L; ++b) eri[a * L * L + b] += B[a] * B[b];
  }
}

struct Spec {
  int L, N, twoS, D;
};

bool ok(sadmrg_ctx* c, int rc, const char* what) {
  if (rc < 0) {
    std::printf("FAIL %s: %d %s\n", what, rc, c ? sadmrg_last_error(c) : "");
    return false;
  }
  return true;
}

}  // namespace

int main(int argc, char** argv) {
  bool block = true, inject = true;
  for (int a = 1; a < argc; ++a) {
    block = block && std::string(argv[a]) != "--no-block";
    inject = inject && std::string(argv[a]) != "--no-inject";
  }
  const std::vector<Spec> specs = {{6, 6, 0, 16}, {7, 6, 2, 20}, {8, 8, 0, 24}, {6, 4, 0, 12}, {7, 8, 2, 20}};
  const int n = (int)specs.size();
  std::vector<sadmrg_ctx*> ctx(n, nullptr), twin(n, nullptr);
  std::vector<int> Ds;
  auto make_spec = [&](const Spec& s, int k, sadmrg_ctx** out) -> bool {
    std::vector<int> irr(s.L, 0);
    if (!ok(nullptr, sadmrg_create(out, s.L, 1, irr.data(), 0), "create")) return false;
    std::vector<double> h, eri;
    integrals(s.L, 11 + k, h, eri);
    return ok(*out, sadmrg_set_integrals(*out, 0.0, h.data(), eri.data(), 1e-10), "integrals") &&
           ok(*out, sadmrg_set_target(*out, s.N, s.twoS, 0), "target") &&
           ok(*out, sadmrg_set_davidson(*out, 1e-8, 16, 80), "davidson") &&
           ok(*out, sadmrg_set_seed(*out, 5 + k), "seed");
  };
  auto make = [&](int k, sadmrg_ctx** out) -> bool { return make_spec(specs[k], k, out); };
  for (int k = 0; k < n; ++k) {
    if (!make(k, &ctx[k]) || !make(k, &twin[k])) return 1;
    if (!ok(ctx[k], sadmrg_init_mps(ctx[k], specs[k].D), "init")) return 1;
    Ds.push_back(specs[k].D);
  }
  std::vector<double> e(n), st(16);
  // FP64 lockstep sweeps (worker threads prepare and update the problems)
  for (int s = 0; s < 2; ++s)
    if (!ok(ctx[0], sadmrg_batch_sweep(ctx.data(), n, Ds.data(), e.data(), st.data()), "batch sweep")) return 1;
  // the same next sweep in lockstep and one problem at a time must agree
  std::vector<std::vector<char>> blobs(n);
  for (int k = 0; k < n; ++k) {
    size_t bytes = 0;
    if (!ok(ctx[k], sadmrg_mps_export(ctx[k], nullptr, &bytes), "export size")) return 1;
    blobs[k].resize(bytes);
    if (!ok(ctx[k], sadmrg_mps_export(ctx[k], blobs[k].data(), &bytes), "export")) return 1;
    if (!ok(twin[k], sadmrg_mps_import(twin[k], blobs[k].data(), bytes), "import")) return 1;
  }
  if (!ok(ctx[0], sadmrg_batch_sweep(ctx.data(), n, Ds.data(), e.data(), st.data()), "batch sweep")) return 1;
  double worst = 0.0;
  for (int k = 0; k < n; ++k) {
    double es = 0.0;
    if (!ok(twin[k], sadmrg_sweep(twin[k], Ds[k], &es), "sweep")) return 1;
    worst = std::fmax(worst, std::fabs(es - e[k]));
  }
  // mixed precision and checkpointed blocks in lockstep
  for (int k = 0; k < n; ++k) {
    if (!ok(ctx[k], sadmrg_set_precision(ctx[k], 1, 1e-5), "precision")) return 1;
    if (!ok(ctx[k], sadmrg_set_block_checkpoints(ctx[k], 2), "checkpoints")) return 1;
  }
  if (!ok(ctx[0], sadmrg_batch_sweep(ctx.data(), n, Ds.data(), e.data(), st.data()), "mixed batch sweep")) return 1;
  // the energy adjoint of each problem
  for (int k = 0; k < n; ++k) {
    const int L = specs[k].L;
    std::vector<double> g1((size_t)L * L), g2((size_t)L * L * L * L);
    double er = 0.0;
    if (!ok(ctx[k], sadmrg_rdm(ctx[k], g1.data(), g2.data(), &er), "rdm")) return 1;
    double tr = 0.0;
    for (int i = 0; i < L; ++i) tr += g1[(size_t)i * L + i];
    if (std::fabs(tr - specs[k].N) > 1e-8) {
      std::printf("FAIL trace of the 1-RDM %g against N = %d\n", tr, specs[k].N);
      return 1;
    }
  }
  // injected device errors -- a gather inside the batch's worker threads or
  // a plain sweep (beside its planning thread), a GEMM launch of a shared
  // sigma or of one context's -- come back as errors of the call, and the
  // contexts work again from a fresh MPS (a lockstep sweep and a separate one)
  struct Inject {
    std::atomic<int>* counter;
    int nth;  // the launch that fails, counted from the start of the call
    bool batch;
    const char* what;
  };
  const std::vector<Inject> injects = {{&sadmrg::emu_fail_gathers, 1, true, "gather in a batch"},
                                      {&sadmrg::emu_fail_gathers, 5, false, "gather in a sweep"},
                                      {&sadmrg::emu_fail_gemms, 40, true, "GEMM in a batch"},
                                      {&sadmrg::emu_fail_gemms, 25, false, "GEMM in a sweep"}};
  for (const Inject& q : inject ? injects : std::vector<Inject>()) {
    for (int k = 0; k < n; ++k)
      if (!ok(ctx[k], sadmrg_init_mps(ctx[k], Ds[k]), "init before injection")) return 1;
    *q.counter = q.nth;
    const int rc_fail = q.batch ? sadmrg_batch_sweep(ctx.data(), n, Ds.data(), e.data(), st.data())
                                : sadmrg_sweep(ctx[0], Ds[0], &e[0]);
    const bool injected = q.counter->load() <= 0;
    *q.counter = 0;
    if (rc_fail >= 0 || !injected) {
      std::printf("FAIL injected %s: rc %d, injected %d\n", q.what, rc_fail, (int)injected);
      return 1;
    }
    for (int k = 0; k < n; ++k)
      if (!ok(ctx[k], sadmrg_init_mps(ctx[k], Ds[k]), "init after failure")) return 1;
    if (!ok(ctx[0], sadmrg_batch_sweep(ctx.data(), n, Ds.data(), e.data(), st.data()), "batch sweep after failure") ||
        !ok(ctx[1], sadmrg_sweep(ctx[1], Ds[1], &e[1]), "sweep after failure"))
      return 1;
  }
  // misuse of the C ABI is refused with EINVAL and leaves the context usable
  if (inject) {
    sadmrg_ctx* u = nullptr;
    if (!make(0, &u)) return 1;
    std::vector<char> junk(64, 7);
    size_t jb = 0;
    const int D0 = specs[0].D;
    const int rcs[] = {sadmrg_sweep(u, D0, &e[0]),               // no MPS yet
                       sadmrg_init_mps(u, 0),                    // D < 1
                       sadmrg_set_target(u, -2, 0, 0),           // N < 0
                       sadmrg_set_precision(u, 7, 1e-5),         // no such mode
                       sadmrg_mps_import(u, junk.data(), junk.size()),  // not an MPS blob
                       sadmrg_mps_export(u, nullptr, &jb),       // no two-site centre
                       sadmrg_batch_sweep(nullptr, 1, &D0, nullptr, nullptr)};
    for (int rc : rcs)
      if (rc >= 0) {
        std::printf("FAIL misuse accepted (rc %d)\n", rc);
        return 1;
      }
    double eu = 0.0;
    if (!ok(u, sadmrg_init_mps(u, D0), "init after misuse") || !ok(u, sadmrg_sweep(u, D0, &eu), "sweep after misuse"))
      return 1;
    sadmrg_destroy(u);
  }
  for (int k = 0; k < n; ++k) {
    sadmrg_destroy(ctx[k]);
    sadmrg_destroy(twin[k]);
  }
  // the decomposition of sectors with 64 or more singular values (the first
  // six steps of a larger problem after one sweep of short Davidson solves):
  // the block path and the one-workgroup path give the same micro-iterations
  double svd_diff = 0.0;
  long block_pairs = 0;
  if (block) {
    const Spec big = {10, 10, 0, 200};
    sadmrg_ctx *w = nullptr, *w2 = nullptr;
    double ew = 0.0;
    if (!make_spec(big, 7, &w) || !make_spec(big, 7, &w2)) return 1;
    for (sadmrg_ctx* c : {w, w2})
      if (!ok(c, sadmrg_set_davidson(c, 1e-8, 8, 2), "davidson")) return 1;
    if (!ok(w, sadmrg_init_mps(w, big.D), "init") || !ok(w, sadmrg_sweep(w, big.D, &ew), "sweep")) return 1;
    size_t bytes = 0;
    if (!ok(w, sadmrg_mps_export(w, nullptr, &bytes), "export size")) return 1;
    std::vector<char> blob(bytes);
    if (!ok(w, sadmrg_mps_export(w, blob.data(), &bytes), "export") ||
        !ok(w2, sadmrg_mps_import(w2, blob.data(), bytes), "import") ||
        !ok(w, sadmrg_mps_import(w, blob.data(), bytes), "import"))
      return 1;
    sadmrg::emu_svd_block_off = true;
    if (!ok(w2, sadmrg_advance(w2, big.D, 6, &ew), "advance")) return 1;
    sadmrg::emu_svd_block_off = false;
    const long before = sadmrg::emu_svd_block_pairs_run;
    if (!ok(w, sadmrg_advance(w, big.D, 6, &ew), "advance")) return 1;
    block_pairs = sadmrg::emu_svd_block_pairs_run - before;
    int n1 = 0, n2 = 0;
    sadmrg_get_trace(w, nullptr, &n1);
    sadmrg_get_trace(w2, nullptr, &n2);
    std::vector<double> t1(std::max(n1, 1)), t2(std::max(n2, 1));
    sadmrg_get_trace(w, t1.data(), &n1);
    sadmrg_get_trace(w2, t2.data(), &n2);
    for (int q = 1; q <= 6; ++q)
      svd_diff = std::fmax(svd_diff, q <= n1 && q <= n2 ? std::fabs(t1[n1 - q] - t2[n2 - q]) : 1.0);
    sadmrg_destroy(w2);
    sadmrg_destroy(w);
  }
  std::printf("emulated batch: %d problems, lockstep vs separate max |dE| %.3e; block decomposition: %ld block "
              "pairs, against one workgroup |dE| %.3e\n",
              n, worst, block_pairs, svd_diff);
  return worst <= 1e-8 && (!block || block_pairs > 0) && svd_diff <= 1e-9 ? 0 : 2;
}
