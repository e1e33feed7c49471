// Host-layer checks of libtlda run under AddressSanitizer and
// UndefinedBehaviorSanitizer (the library's host code is instrumented; device
// code is not).  Covered: status strings, configuration checks of
// tlda_create, argument checks of the batch, staging, step, encoder, plan,
// graph and checkpoint calls, the encoder's parameter round trip, a short
// moments -> refresh -> step sequence through the staging
// slots, and the checkpoint loader fed truncations of a valid checkpoint and
// checkpoints with corrupted header fields.
//
// Usage: host_abi_check cpu   (calls that need no device; tlda_create must
//                              fail cleanly without one)
//        host_abi_check gpu   (a context on the current device)
// Exit status 0 when every expectation holds; a sanitizer report ends the
// process with a non-zero status on its own.
#include <hip/hip_runtime_api.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "tlda.h"

static int g_failures = 0;

#define EXPECT(cond)                                                    \
  do {                                                                  \
    if (!(cond)) {                                                      \
      std::fprintf(stderr, "FAILED %s:%d: %s\n", __FILE__, __LINE__, #cond); \
      ++g_failures;                                                     \
    }                                                                   \
  } while (0)

static tlda_config base_config(int V, int K, int D) {
  tlda_config c;
  std::memset(&c, 0, sizeof(c));
  c.V = V;
  c.K = K;
  c.D = D;
  c.alpha0 = 1.0;
  c.theta = 0.0;
  c.eig_iters = 40;
  c.eig_seed = 7;
  return c;
}

static void check_status_strings() {
  for (int s = 0; s <= 9; ++s) {
    const char* m = tlda_status_str(static_cast<tlda_status>(s));
    EXPECT(m != nullptr && std::strlen(m) > 0);
  }
}

// Configurations tlda_create must refuse before it touches a device.
static void check_bad_configs() {
  tlda_ctx* ctx = reinterpret_cast<tlda_ctx*>(0x1);
  tlda_config c = base_config(100, 8, 8);
  EXPECT(tlda_create(nullptr, nullptr, &ctx) == TLDA_ERR_ARG);
  EXPECT(tlda_create(&c, nullptr, nullptr) == TLDA_ERR_ARG);
  struct Bad {
    void (*edit)(tlda_config&);
    tlda_status want;
  };
  const Bad bad[] = {
      {[](tlda_config& x) { x.alpha0 = 0.0; }, TLDA_ERR_ARG},
      {[](tlda_config& x) { x.alpha0 = -1.0; }, TLDA_ERR_ARG},
      {[](tlda_config& x) { x.theta = -0.5; }, TLDA_ERR_ARG},
      {[](tlda_config& x) { x.flags = 0x100; }, TLDA_ERR_ARG},
      {[](tlda_config& x) { x.eig_iters = -1; }, TLDA_ERR_ARG},
      {[](tlda_config& x) { x.V = 2; }, TLDA_ERR_SHAPE},
      {[](tlda_config& x) { x.V = 131073; }, TLDA_ERR_SHAPE},
      {[](tlda_config& x) { x.K = 0; }, TLDA_ERR_SHAPE},
      {[](tlda_config& x) { x.D = 0; }, TLDA_ERR_SHAPE},
      {[](tlda_config& x) { x.D = 101; }, TLDA_ERR_SHAPE},
      {[](tlda_config& x) { x.V = 100000; x.D = 200; x.K = 100; }, TLDA_ERR_SHAPE},
      {[](tlda_config& x) { x.eig_block = 4; }, TLDA_ERR_SHAPE},
      {[](tlda_config& x) { x.flags = TLDA_BF16; x.V = 300; x.D = 200; }, TLDA_ERR_SHAPE},
  };
  for (const Bad& b : bad) {
    tlda_config x = base_config(100, 8, 8);
    b.edit(x);
    ctx = reinterpret_cast<tlda_ctx*>(0x1);
    EXPECT(tlda_create(&x, nullptr, &ctx) == b.want);
    EXPECT(ctx == nullptr);
  }
  EXPECT(tlda_mlp_param_count(16, 32, 8) > 0);
}

// Null and out-of-range arguments on a live context: refused with a message.
static void check_bad_arguments(tlda_ctx* ctx) {
  EXPECT(tlda_update_moments(nullptr, nullptr, 0) == TLDA_ERR_ARG);
  tlda_csr_batch b;
  std::memset(&b, 0, sizeof(b));
  b.n_rows = 4;
  b.slot = -1;
  EXPECT(tlda_update_moments(ctx, &b, 0) != TLDA_OK);          // NULL row_ptr
  EXPECT(std::strlen(tlda_last_error(ctx)) > 0);
  b.n_rows = -1;
  EXPECT(tlda_update_moments(ctx, &b, 0) != TLDA_OK);
  EXPECT(tlda_update_moments(ctx, nullptr, 0x40) != TLDA_OK);   // unknown flag
  tlda_csr_batch out;
  std::memset(&out, 0, sizeof(out));
  EXPECT(tlda_stage_batch(ctx, nullptr, 0, &out) == TLDA_ERR_ARG);
  tlda_csr_batch h;
  std::memset(&h, 0, sizeof(h));
  h.n_rows = 1;
  EXPECT(tlda_stage_batch(ctx, &h, 2, &out) == TLDA_ERR_ARG);  // bad slot
  EXPECT(tlda_stage_batch(ctx, &h, 0, &out) == TLDA_ERR_ARG);  // NULL row_ptr
  h.n_rows = -3;
  EXPECT(tlda_stage_batch(ctx, &h, 0, &out) == TLDA_ERR_SHAPE);
  float phi[64] = {0};
  EXPECT(tlda_whiten_cp_step(ctx, nullptr, 0.1f, phi, nullptr, nullptr, nullptr) != TLDA_OK);
  EXPECT(tlda_save_state(ctx, nullptr, nullptr) != TLDA_OK);
  unsigned char junk[8] = {0};
  EXPECT(tlda_load_state(ctx, junk, sizeof(junk)) != TLDA_OK);
  EXPECT(tlda_load_state(ctx, nullptr, 100) != TLDA_OK);
}

// A small corpus staged from pinned host memory: moments, a refresh, a step;
// then the checkpoint round trip, every truncation and corrupted headers.
static void check_sequence(tlda_ctx* ctx, int V, int K, int D) {
  const int n = 300;
  std::vector<int32_t> rp(n + 1, 0), ci;
  std::vector<float> va;
  unsigned s = 12345u;
  auto rnd = [&]() { s = s * 1664525u + 1013904223u; return s >> 8; };
  for (int r = 0; r < n; ++r) {
    const int len = 3 + static_cast<int>(rnd() % 20);
    int col = static_cast<int>(rnd() % 7);
    for (int t = 0; t < len && col < V; ++t) {
      ci.push_back(col);
      va.push_back(static_cast<float>(1 + rnd() % 3));
      col += 1 + static_cast<int>(rnd() % 9);
    }
    rp[r + 1] = static_cast<int32_t>(ci.size());
  }
  const int nnz = static_cast<int>(ci.size());
  int32_t* hrp = nullptr;
  int32_t* hci = nullptr;
  float* hva = nullptr;
  EXPECT(hipHostMalloc(reinterpret_cast<void**>(&hrp), (n + 1) * sizeof(int32_t), 0) == hipSuccess);
  EXPECT(hipHostMalloc(reinterpret_cast<void**>(&hci), nnz * sizeof(int32_t), 0) == hipSuccess);
  EXPECT(hipHostMalloc(reinterpret_cast<void**>(&hva), nnz * sizeof(float), 0) == hipSuccess);
  if (!hrp || !hci || !hva) return;
  std::memcpy(hrp, rp.data(), (n + 1) * sizeof(int32_t));
  std::memcpy(hci, ci.data(), nnz * sizeof(int32_t));
  std::memcpy(hva, va.data(), nnz * sizeof(float));
  tlda_csr_batch h;
  std::memset(&h, 0, sizeof(h));
  h.n_rows = n;
  h.nnz = nnz;
  h.row_ptr = hrp;
  h.col_idx = hci;
  h.val = hva;
  h.first_doc = 1000;
  tlda_csr_batch dev;
  EXPECT(tlda_stage_batch(ctx, &h, 0, &dev) == TLDA_OK);
  EXPECT(tlda_update_moments(ctx, &dev, TLDA_REFRESH_W) == TLDA_OK);
  float* phi = nullptr;
  EXPECT(hipMalloc(reinterpret_cast<void**>(&phi), sizeof(float) * D * K) == hipSuccess);
  std::vector<float> phi0(D * K, 0.0f);
  for (int i = 0; i < D && i < K; ++i) phi0[i * K + i] = 0.5f;
  EXPECT(hipMemcpy(phi, phi0.data(), sizeof(float) * D * K, hipMemcpyHostToDevice) == hipSuccess);
  EXPECT(tlda_stage_batch(ctx, &h, 1, &dev) == TLDA_OK);
  EXPECT(tlda_whiten_cp_step(ctx, &dev, 1e-3f, phi, nullptr, nullptr, nullptr) == TLDA_OK);
  EXPECT(hipDeviceSynchronize() == hipSuccess);

  size_t len = 0;
  EXPECT(tlda_save_state(ctx, nullptr, &len) == TLDA_OK);
  EXPECT(len > 64);
  std::vector<unsigned char> ck(len);
  EXPECT(tlda_save_state(ctx, ck.data(), &len) == TLDA_OK);
  EXPECT(tlda_load_state(ctx, ck.data(), len) == TLDA_OK);
  // truncations (every length below 256 bytes, then every 97th), each in a
  // buffer of exactly that size (a read past it is a heap overflow for the
  // sanitizer)
  for (size_t cut = 0; cut < len; cut += (cut < 256 ? 1 : 97)) {
    std::vector<unsigned char> part(ck.begin(), ck.begin() + cut);
    EXPECT(tlda_load_state(ctx, cut ? part.data() : ck.data(), cut) != TLDA_OK);
  }
  // corrupted header words: refused or accepted, never a read out of bounds
  for (size_t off = 0; off < 64 && off + 4 <= len; off += 4) {
    std::vector<unsigned char> bad(ck);
    const uint32_t flip = 0x7fffffffu;
    std::memcpy(bad.data() + off, &flip, 4);
    (void)tlda_load_state(ctx, bad.data(), bad.size());
  }
  EXPECT(tlda_load_state(ctx, ck.data(), len) == TLDA_OK);
  // a context of another shape refuses the checkpoint
  tlda_config other = base_config(V, K, D > 1 ? D - 1 : 1);
  tlda_ctx* ctx2 = nullptr;
  EXPECT(tlda_create(&other, nullptr, &ctx2) == TLDA_OK);
  if (ctx2) {
    EXPECT(tlda_load_state(ctx2, ck.data(), len) == TLDA_ERR_SHAPE);
    tlda_destroy(ctx2);
  }
  hipFree(phi);
  hipHostFree(hrp);
  hipHostFree(hci);
  hipHostFree(hva);
}

// The encoder's host calls: shape checks, and a parameter round trip
// through host buffers of exactly the parameter count.
static void check_mlp(bool gpu) {
  EXPECT(tlda_mlp_param_count(0, 32, 8) == 0);
  tlda_mlp* m = reinterpret_cast<tlda_mlp*>(0x1);
  EXPECT(tlda_mlp_create(16, 32, 8, 64, nullptr, nullptr) == TLDA_ERR_ARG);
  EXPECT(tlda_mlp_create(0, 32, 8, 64, nullptr, &m) == TLDA_ERR_SHAPE);
  EXPECT(m == nullptr);
  EXPECT(tlda_mlp_create(16, TLDA_MLP_MAX_WIDTH + 1, 8, 64, nullptr, &m) == TLDA_ERR_SHAPE);
  EXPECT(tlda_mlp_create(16, 32, TLDA_MAX_K + 1, 64, nullptr, &m) == TLDA_ERR_SHAPE);
  EXPECT(tlda_mlp_create(16, 32, 8, 0, nullptr, &m) == TLDA_ERR_SHAPE);
  if (!gpu) return;
  EXPECT(tlda_mlp_create(16, 32, 8, 64, nullptr, &m) == TLDA_OK);
  if (!m) return;
  const int64_t np = tlda_mlp_param_count(16, 32, 8);
  std::vector<float> p(np), q(np, -1.0f);
  for (int64_t i = 0; i < np; ++i) p[i] = 0.001f * static_cast<float>(i % 997);
  EXPECT(tlda_mlp_set_params(m, p.data()) == TLDA_OK);
  EXPECT(tlda_mlp_get_params(m, q.data()) == TLDA_OK);
  EXPECT(std::memcmp(p.data(), q.data(), np * sizeof(float)) == 0);
  EXPECT(tlda_mlp_set_params(m, nullptr) != TLDA_OK);
  EXPECT(tlda_mlp_forward(m, nullptr, 4, nullptr) != TLDA_OK);
  EXPECT(std::strlen(tlda_mlp_last_error(m)) > 0);
  tlda_mlp_destroy(m);
  tlda_mlp_destroy(nullptr);
}

// Multi-slice plans and graph capture refuse malformed requests.
static void check_plans(tlda_ctx* ctx) {
  tlda_multi* plan = reinterpret_cast<tlda_multi*>(0x1);
  EXPECT(tlda_multi_create(0, &ctx, nullptr, nullptr, nullptr, nullptr, &plan) == TLDA_ERR_ARG);
  EXPECT(plan == nullptr);
  tlda_csr_batch b;
  std::memset(&b, 0, sizeof(b));
  b.slot = -1;
  float* phis[1] = {reinterpret_cast<float*>(0x100)};
  const float betas[1] = {0.1f};
  tlda_ctx* none[1] = {nullptr};
  EXPECT(tlda_multi_create(1, none, &b, phis, betas, nullptr, &plan) == TLDA_ERR_ARG);
  // an FP32 context is not a multi-slice shape (BF16 only)
  EXPECT(tlda_multi_create(1, &ctx, &b, phis, betas, nullptr, &plan) != TLDA_OK);
  EXPECT(plan == nullptr);
  tlda_multi_destroy(nullptr);
  tlda_graph* g = reinterpret_cast<tlda_graph*>(0x1);
  EXPECT(tlda_graph_capture_steps(ctx, nullptr, 1, 0.1f, phis[0], &g) == TLDA_ERR_ARG);
  EXPECT(g == nullptr);
  EXPECT(tlda_graph_capture_steps(ctx, &b, 0, 0.1f, phis[0], &g) == TLDA_ERR_ARG);
  EXPECT(tlda_graph_capture(nullptr, 1, &g) != TLDA_OK);
  tlda_graph_destroy(nullptr);
}

int main(int argc, char** argv) {
  const bool gpu = argc > 1 && std::strcmp(argv[1], "gpu") == 0;
  check_status_strings();
  check_bad_configs();
  check_mlp(gpu);
  const int V = 200, K = 8, D = 8;
  tlda_config c = base_config(V, K, D);
  tlda_ctx* ctx = nullptr;
  const tlda_status st = tlda_create(&c, nullptr, &ctx);
  if (!gpu) {
    // without a device the context cannot be made, and nothing is leaked
    EXPECT(st == TLDA_ERR_DEVICE || st == TLDA_OK);
    if (ctx) tlda_destroy(ctx);
  } else {
    EXPECT(st == TLDA_OK);
    if (ctx) {
      check_bad_arguments(ctx);
      check_plans(ctx);
      check_sequence(ctx, V, K, D);
      tlda_destroy(ctx);
    }
  }
  tlda_destroy(nullptr);
  std::printf("host_abi_check %s: %d failed expectations\n", gpu ? "gpu" : "cpu", g_failures);
  return g_failures == 0 ? 0 : 1;
}
