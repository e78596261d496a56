// Drives the library's host runtime against the HIP stub (hip_stub.cpp) under the sanitizers:
// pass planning and workspace layouts over many shapes, the FP64 utilities, every argument and
// allocation error path of problem creation, and the call sequences of the host, device-pointer and
// allocation-free entry points.  The kernels do nothing here, so only the host code is exercised;
// results are not checked, memory safety and the returned statuses are.  Exits non-zero on failure.
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include "../../include/qhvp.h"
#include "../../paper_2604_20384_amd/csrc/qhvp_internal.h"

extern "C" void stub_fail_allocations(int device_calls, int pinned_calls);
extern "C" void stub_fail_pinned_nth(int nth);
extern "C" long stub_live_blocks();
extern "C" int hipMalloc(void** ptr, size_t size);   // from the stub (hipError_t is an int enum)
extern "C" int hipFree(void* ptr);

static int g_fail = 0;
#define CHECK(cond)                                                                   \
  do {                                                                                \
    if (!(cond)) {                                                                    \
      std::fprintf(stderr, "FAILED %s:%d: %s (%s)\n", __FILE__, __LINE__, #cond, qhvp_last_error()); \
      ++g_fail;                                                                       \
    }                                                                                 \
  } while (0)

using cd = std::complex<double>;
static std::mt19937_64 rng(7);
static std::vector<double> random_gates(int K, bool unitary) {
  std::normal_distribution<double> nd;
  std::vector<double> g((size_t)K * 32);
  for (auto& x : g) x = nd(rng);
  if (unitary) {   // polar factor through the library's retraction at 0: R_A(0) of a random A
    std::vector<double> z(g.size(), 0.0), u(g.size());
    if (qhvp_retract(K, g.data(), z.data(), u.data()) == QHVP_OK) return u;
  }
  return g;
}

// The layer arithmetic the translationally invariant kernels use, against the brickwall's gates
// enumerated layer by layer (App. E's layer sets).
static void ti_layers() {
  for (int n = 2; n <= 30; ++n)
    for (int L : {1, 2, 3, 4, 7, 20, 41}) {
      int k = 0;
      for (int l = 0; l < L; ++l) {
        CHECK(qhvp::ti_first_gate(l, n) == k);
        int cnt = 0;
        for (int q = l % 2; q + 1 < n; q += 2, ++k, ++cnt) CHECK(qhvp::ti_layer_of(k, n) == l);
        CHECK(qhvp::ti_gate_count(l, n) == cnt);
      }
      CHECK(k == qhvp_num_gates(n, L));
    }
  std::puts("OK ti layers");
}

static void plans() {
  for (int n = 2; n <= 24; ++n)
    for (int L : {1, 2, 3, 5, 8, 13, 20, 32, 40}) {
      const int K = qhvp_num_gates(n, L);
      const int np = qhvp_plan(n, L, 0, nullptr, nullptr);
      CHECK(K > 0 && np > 0);
      std::vector<int> per(np), order(K), seen(K, 0);
      CHECK(qhvp_plan(n, L, np, per.data(), order.data()) == np);
      int sum = 0;
      for (int c : per) { CHECK(c >= 1 && c <= 6); sum += c; }
      CHECK(sum == K);
      for (int k : order) { CHECK(k >= 0 && k < K); if (k >= 0 && k < K) seen[k]++; }
      for (int s : seen) CHECK(s == 1);
      CHECK(qhvp_plan(n, L, np - 1, per.data(), nullptr) < 0);   // too small a buffer
      for (int prec : {0, 1})
        for (int ck : {0, 1, 2, 4, -2, QHVP_CKPT_REBUILD})
          CHECK(qhvp_workspace_bytes(n, L, 2 * L, 3, (qhvp_precision)prec, ck, 1) > 0);
      // rebuilding keeps two slots of states, keeping every boundary one per pass
      if (np >= 2)
        CHECK(qhvp_workspace_bytes(n, L, 2 * L, 3, QHVP_C64_ACC64, QHVP_CKPT_REBUILD, 1) <=
              qhvp_workspace_bytes(n, L, 2 * L, 3, QHVP_C64_ACC64, 0, 1));
    }
  CHECK(qhvp_plan(1, 3, 0, nullptr, nullptr) < 0 && qhvp_plan(31, 3, 0, nullptr, nullptr) < 0);
  CHECK(qhvp_workspace_bytes(1, 3, 6, 3, QHVP_C64_ACC64, 0, 1) == 0);
  CHECK(qhvp_workspace_bytes(6, 0, 6, 3, QHVP_C64_ACC64, 0, 1) == 0);
  CHECK(qhvp_workspace_bytes(6, 3, 6, 0, QHVP_C64_ACC64, 0, 1) == 0);
  CHECK(qhvp_workspace_bytes(6, 3, 6, 3, (qhvp_precision)7, 0, 1) == 0);
  std::puts("OK plans");
}

static void utilities() {
  const int K = 9;
  auto G = random_gates(K, true);
  CHECK(qhvp_unitarity_error(K, G.data()) < 1e-12);
  auto X = random_gates(K, false);
  std::vector<double> P(X.size()), PP(X.size()), R(X.size()), H(X.size());
  CHECK(qhvp_project(K, G.data(), X.data(), P.data()) == QHVP_OK);
  CHECK(qhvp_project(K, G.data(), P.data(), PP.data()) == QHVP_OK);
  double d = 0;
  for (size_t i = 0; i < P.size(); ++i) d = std::max(d, std::abs(P[i] - PP[i]));
  CHECK(d < 1e-12);   // idempotent
  CHECK(qhvp_riemannian_hvp(K, G.data(), X.data(), X.data(), P.data(), H.data()) == QHVP_OK);
  CHECK(qhvp_retract(K, G.data(), P.data(), R.data()) == QHVP_OK);
  CHECK(qhvp_unitarity_error(K, R.data()) < 1e-10);
  CHECK(qhvp_project(0, nullptr, nullptr, nullptr) == QHVP_ERR_INVALID);
  CHECK(qhvp_retract(K, nullptr, P.data(), R.data()) == QHVP_ERR_INVALID);
  std::puts("OK utilities");
}

static void creation_errors() {
  qhvp_ctx* ctx = nullptr;
  CHECK(qhvp_ctx_create(5, &ctx) == QHVP_ERR_INVALID);
  CHECK(qhvp_ctx_create(0, &ctx) == QHVP_OK && ctx);
  const long live0 = stub_live_blocks();
  const int n = 8, L = 4, Lr = 8, ns = 3;
  auto uref = random_gates(qhvp_num_gates(n, Lr), true);
  std::vector<double> samples((size_t)ns * n * 4, 0.5);
  qhvp_problem* p = nullptr;
  // shapes and arguments
  CHECK(qhvp_problem_create(ctx, 1, L, Lr, uref.data(), samples.data(), ns, QHVP_C64_ACC64, 0, 1, nullptr, 0, nullptr, &p) == QHVP_ERR_INVALID);
  CHECK(qhvp_problem_create(ctx, n, L, Lr, nullptr, samples.data(), ns, QHVP_C64_ACC64, 0, 1, nullptr, 0, nullptr, &p) == QHVP_ERR_INVALID);
  std::vector<double> bad = samples;
  bad[3] = NAN;
  CHECK(qhvp_problem_create(ctx, n, L, Lr, uref.data(), bad.data(), ns, QHVP_C64_ACC64, 0, 1, nullptr, 0, nullptr, &p) == QHVP_ERR_INVALID);
  // a caller workspace that is too small, and one that is misaligned
  const size_t need = qhvp_workspace_bytes(n, L, Lr, ns, QHVP_C64_ACC64, 0, 1);
  void* ws = nullptr;
  CHECK(hipMalloc(&ws, need + 512) == 0);
  CHECK(qhvp_problem_create(ctx, n, L, Lr, uref.data(), samples.data(), ns, QHVP_C64_ACC64, 0, 1, ws, need - 1, nullptr, &p) == QHVP_ERR_NOMEM);
  CHECK(qhvp_problem_create(ctx, n, L, Lr, uref.data(), samples.data(), ns, QHVP_C64_ACC64, 0, 1, (char*)ws + 8, need, nullptr, &p) == QHVP_ERR_INVALID);
  // allocation failures: the library's own workspace, then its pinned staging
  stub_fail_allocations(1, 0);
  CHECK(qhvp_problem_create(ctx, n, L, Lr, uref.data(), samples.data(), ns, QHVP_C64_ACC64, 0, 1, nullptr, 0, nullptr, &p) == QHVP_ERR_NOMEM);
  CHECK(std::string(qhvp_last_error()).find("hipMalloc") != std::string::npos);
  for (int k = 1; k <= 3; ++k) {   // the 1st, 2nd or 3rd pinned buffer fails (a fresh context: nothing pooled)
    qhvp_ctx* c2 = nullptr;
    CHECK(qhvp_ctx_create(0, &c2) == QHVP_OK);
    const long before = stub_live_blocks();
    stub_fail_pinned_nth(k);
    CHECK(qhvp_problem_create(c2, n, L, Lr, uref.data(), samples.data(), ns, QHVP_C64_ACC64, 0, 1, nullptr, 0, nullptr, &p) == QHVP_ERR_NOMEM);
    CHECK(std::string(qhvp_last_error()).find("pinned") != std::string::npos);
    stub_fail_pinned_nth(0);
    qhvp_ctx_destroy(c2);             // frees what the failed creation returned to the pool
    CHECK(stub_live_blocks() == before);
  }
  stub_fail_allocations(0, 0);
  CHECK(hipFree(ws) == 0);
  CHECK(stub_live_blocks() == live0);
  qhvp_ctx_destroy(ctx);
  std::puts("OK creation errors");
}

static void call_sequences() {
  qhvp_ctx* ctx = nullptr;
  CHECK(qhvp_ctx_create(0, &ctx) == QHVP_OK);
  const long live0 = stub_live_blocks();
  for (int prec : {0, 1})
    for (int ck : {0, 1, -2, QHVP_CKPT_REBUILD}) {
      const int n = 7, L = 5, Lr = 10, ns = 4;
      const int K = qhvp_num_gates(n, L);
      auto uref = random_gates(qhvp_num_gates(n, Lr), true);
      std::vector<double> samples((size_t)ns * n * 4, 0.25);
      qhvp_problem* p = nullptr;
      CHECK(qhvp_problem_create(ctx, n, L, Lr, uref.data(), samples.data(), ns, (qhvp_precision)prec, ck, 1, nullptr, 0, nullptr, &p) == QHVP_OK);
      if (!p) continue;
      auto G = random_gates(K, true), V = random_gates(K, false);
      std::vector<double> g((size_t)K * 32), h((size_t)K * 32), T((size_t)ns * 2), Om((size_t)ns * 2);
      double c = 0, F = 0;
      CHECK(qhvp_set_profiling(p, 1) == QHVP_OK);
      CHECK(qhvp_cost(p, G.data(), &c, &F) == QHVP_OK);
      CHECK(qhvp_grad(p, G.data(), QHVP_RIEMANNIAN, &c, &F, g.data()) == QHVP_OK);
      CHECK(qhvp_hvp(p, G.data(), V.data(), QHVP_EUCLIDEAN, &c, &F, g.data(), h.data()) == QHVP_OK);
      CHECK(qhvp_forward(p, G.data(), V.data(), QHVP_RIEMANNIAN, &c, &F) == QHVP_OK);
      CHECK(qhvp_backward(p, g.data(), h.data()) == QHVP_OK);
      CHECK(qhvp_backward(p, g.data(), h.data()) == QHVP_ERR_INVALID);   // consumed
      std::vector<double> Vs(V.size() * 3);
      for (int m = 0; m < 3; ++m) std::memcpy(&Vs[V.size() * m], V.data(), V.size() * sizeof(double));
      std::vector<double> hs(Vs.size());
      CHECK(qhvp_hvp_batch(p, G.data(), 3, Vs.data(), QHVP_EUCLIDEAN, &c, g.data(), hs.data()) == QHVP_OK);
      CHECK(qhvp_overlaps(p, T.data(), Om.data()) == QHVP_OK);
      std::vector<double> gl((size_t)L * 32), hl((size_t)L * 32);
      double keep_ti = 0;
      auto Gl0 = random_gates(L, true);
      CHECK(qhvp_grad_ti(p, Gl0.data(), QHVP_EUCLIDEAN, &c, &F, gl.data()) == QHVP_OK);
      CHECK(qhvp_hvp_ti(p, Gl0.data(), Gl0.data(), QHVP_RIEMANNIAN, &c, nullptr, gl.data(), hl.data()) == QHVP_OK);
      CHECK(qhvp_hvp_ti(p, Gl0.data(), Gl0.data(), QHVP_EUCLIDEAN, nullptr, nullptr, nullptr, hl.data()) == QHVP_OK);
      auto Gl1 = Gl0;
      Gl1[5] = NAN;
      keep_ti = 2.5;
      CHECK(qhvp_grad_ti(p, Gl1.data(), QHVP_EUCLIDEAN, &keep_ti, nullptr, gl.data()) == QHVP_ERR_INVALID && keep_ti == 2.5);
      CHECK(qhvp_hvp_ti(p, Gl0.data(), nullptr, QHVP_EUCLIDEAN, nullptr, nullptr, nullptr, hl.data()) == QHVP_ERR_INVALID);
      double ms = 0, by = 0, fl = 0;
      long long cnt = 0;
      for (int kind = 0; kind < QHVP_KERNEL_KINDS; ++kind) CHECK(qhvp_kernel_stats(p, kind, &ms, &cnt, &by, &fl) == QHVP_OK);
      int kk = 0, npass = 0, segs = 0;
      size_t wsb = 0;
      CHECK(qhvp_problem_info(p, &kk, &npass, &wsb, &segs) == QHVP_OK && kk == K);
      (void)qhvp_last_device_ms(p);
      (void)qhvp_backward_from_outputs(p);
      (void)qhvp_states_kept_for(p, G.data());
      // errors on the host path: non-finite input, non-unitary Riemannian, NULL outputs
      auto Gb = G;
      Gb[11] = INFINITY;
      double keep = 3.5;
      CHECK(qhvp_hvp(p, Gb.data(), V.data(), QHVP_EUCLIDEAN, &keep, nullptr, nullptr, h.data()) == QHVP_ERR_INVALID && keep == 3.5);
      auto Gn = random_gates(K, false);
      CHECK(qhvp_grad(p, Gn.data(), QHVP_RIEMANNIAN, &keep, nullptr, g.data()) == QHVP_ERR_INVALID && keep == 3.5);
      CHECK(qhvp_hvp(p, G.data(), V.data(), QHVP_EUCLIDEAN, nullptr, nullptr, nullptr, nullptr) == QHVP_ERR_INVALID);
      // device-pointer calls: device buffers from the stub's hipMalloc, and a host pointer refused
      double *dG = nullptr, *dV = nullptr, *dout = nullptr;
      CHECK(hipMalloc((void**)&dG, G.size() * 8) == 0 && hipMalloc((void**)&dV, V.size() * 8) == 0 &&
            hipMalloc((void**)&dout, (2 + 2 * G.size()) * 8) == 0);
      std::memcpy(dG, G.data(), G.size() * 8);
      std::memcpy(dV, V.data(), V.size() * 8);
      CHECK(qhvp_hvp_dev(p, dG, dV, QHVP_EUCLIDEAN, dout, dout + 1, dout + 2, dout + 2 + G.size()) == QHVP_OK);
      CHECK(qhvp_grad_dev(p, dG, QHVP_RIEMANNIAN, dout, nullptr, dout + 2) == QHVP_OK);
      CHECK(qhvp_cost_dev(p, dG, dout, dout + 1) == QHVP_OK);
      CHECK(qhvp_forward_dev(p, dG, dV, QHVP_EUCLIDEAN, nullptr, nullptr) == QHVP_OK);
      CHECK(qhvp_backward_dev(p, dout + 2, dout + 2 + G.size()) == QHVP_OK);
      CHECK(qhvp_hvp_dev(p, G.data(), dV, QHVP_EUCLIDEAN, nullptr, nullptr, nullptr, dout + 2) == QHVP_ERR_INVALID);
      CHECK(qhvp_hvp_dev(p, dG, dV, QHVP_EUCLIDEAN, nullptr, nullptr, nullptr, h.data()) == QHVP_ERR_INVALID);
      double *dGl = nullptr, *dlo = nullptr;
      CHECK(hipMalloc((void**)&dGl, Gl0.size() * 8) == 0 && hipMalloc((void**)&dlo, (2 + 2 * Gl0.size()) * 8) == 0);
      std::memcpy(dGl, Gl0.data(), Gl0.size() * 8);
      CHECK(qhvp_grad_ti_dev(p, dGl, QHVP_RIEMANNIAN, dlo, dlo + 1, dlo + 2) == QHVP_OK);
      CHECK(qhvp_hvp_ti_dev(p, dGl, dGl, QHVP_EUCLIDEAN, nullptr, nullptr, nullptr, dlo + 2 + Gl0.size()) == QHVP_OK);
      CHECK(qhvp_hvp_ti_dev(p, Gl0.data(), dGl, QHVP_EUCLIDEAN, nullptr, nullptr, nullptr, dlo + 2) == QHVP_ERR_INVALID);
      CHECK(qhvp_grad_ti_dev(p, dGl, QHVP_EUCLIDEAN, nullptr, nullptr, gl.data()) == QHVP_ERR_INVALID);
      hipFree(dGl); hipFree(dlo);
      int status = -1;
      CHECK(qhvp_device_status(p, &status) == QHVP_OK);
      // the allocation-free entry point: a small problem runs, a large one is refused
      double *du = nullptr, *ds = nullptr;
      CHECK(hipMalloc((void**)&du, uref.size() * 8) == 0 && hipMalloc((void**)&ds, samples.size() * 8) == 0);
      CHECK(qhvp_hvp_noalloc(ctx, n, L, Lr, du, ds, ns, (qhvp_precision)prec, dG, dV, QHVP_EUCLIDEAN, dout, dout + 1,
                             dout + 2, dout + 2 + G.size(), nullptr) == QHVP_OK);
      CHECK(qhvp_hvp_noalloc(ctx, 24, 2, 2, du, ds, 256, (qhvp_precision)prec, dG, dV, QHVP_EUCLIDEAN, dout, nullptr,
                             nullptr, dout + 2, nullptr) == QHVP_ERR_NOMEM);
      CHECK(qhvp_hvp_noalloc(ctx, n, L, Lr, uref.data(), ds, ns, (qhvp_precision)prec, dG, dV, QHVP_EUCLIDEAN, nullptr,
                             nullptr, nullptr, dout + 2, nullptr) == QHVP_ERR_INVALID);
      hipFree(du); hipFree(ds); hipFree(dG); hipFree(dV); hipFree(dout);
      qhvp_problem_destroy(p);
    }
  qhvp_ctx_destroy(ctx);
  CHECK(stub_live_blocks() <= live0);
  std::puts("OK call sequences");
}

int main() {
  ti_layers();
  plans();
  utilities();
  creation_errors();
  call_sequences();
  if (g_fail) {
    std::printf("%d checks failed\n", g_fail);
    return 1;
  }
  std::puts("ALL OK");
  return 0;
}
