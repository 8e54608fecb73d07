// Drives the C ABI on a host-only context (planning, validation, tuning,
// memory budgets, cost model, argument checks) for the graphs listed in a
// text file, built with AddressSanitizer and UndefinedBehaviorSanitizer.
// Input lines: "qaoa|qaoa64|amp n p m a0 b0 a1 b1 ..." (qaoa64: complex64 only).  Exit status 0 when every
// call returned what its contract states; any sanitizer report aborts.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/qtn.h"

static int g_fail = 0;

#define EXPECT(call, want)                                                                                     \
  do {                                                                                                         \
    const qtn_status s_ = (call);                                                                              \
    if (s_ != (want)) {                                                                                        \
      std::fprintf(stderr, "line %d: %s returned %d, expected %d (%s)\n", __LINE__, #call, (int)s_, (int)(want), \
                   qtn_last_error());                                                                          \
      ++g_fail;                                                                                                \
    }                                                                                                          \
  } while (0)

static void check_plan(qtn_net* net, int m, bool per_edge) {
  EXPECT(qtn_validate_plan(net), QTN_OK);
  qtn_info info;
  EXPECT(qtn_get_info(net, &info), QTN_OK);
  size_t ws = 0, ws1 = 0;
  EXPECT(qtn_workspace_size(net, 0, &ws), QTN_OK);
  EXPECT(qtn_workspace_size(net, 1, &ws1), QTN_OK);
  if (ws == 0 || ws1 < ws) {
    std::fprintf(stderr, "workspace sizes %zu %zu\n", ws, ws1);
    ++g_fail;
  }
  if (per_edge) {
    std::vector<int32_t> w(m), q(m), ni(m), nt(m), nb(m);
    std::vector<double> fb(m), bb(m);
    EXPECT(qtn_cone_stats(net, w.data(), q.data(), ni.data(), nt.data(), nb.data(), fb.data(), bb.data()), QTN_OK);
    for (int e = 0; e < m; ++e)
      if (w[e] < 1 || w[e] > info.max_width || nb[e] < 1) {
        std::fprintf(stderr, "cone %d stats width %d buckets %d\n", e, w[e], nb[e]);
        ++g_fail;
      }
  }
}

static void tunings(qtn_net* net, int m, bool per_edge) {
  qtn_tuning t0, t;
  EXPECT(qtn_get_tuning(net, &t0), QTN_OK);
  const int32_t threads[] = {64, 128, 256, 512};
  const int32_t seq[] = {6, 10, 14, 16};
  for (int k = 0; k < 4; ++k) {
    t = t0;
    t.threads = threads[k];
    t.seq_max_bits = seq[k];
    t.lds_kb = k == 0 ? 0 : 32 * k;
    t.fuse_adjoint = k & 1;
    t.lds_threads = 64 << (k % 3);
    EXPECT(qtn_set_tuning(net, &t), QTN_OK);
    check_plan(net, m, per_edge);
  }
  t = t0;
  t.threads = 100;
  EXPECT(qtn_set_tuning(net, &t), QTN_EINVAL);
  t = t0;
  t.lds_kb = 1000;
  EXPECT(qtn_set_tuning(net, &t), QTN_EINVAL);
  EXPECT(qtn_set_tuning(net, &t0), QTN_OK);
  // tiles per bucket-signature band
  qtn_band_tuning b[QTN_BANDS] = {{19, 64, 8}, {23, 256, 0}, {0, 0, 0}}, got[QTN_BANDS];
  EXPECT(qtn_set_band_tuning(net, b), QTN_OK);
  check_plan(net, m, per_edge);
  EXPECT(qtn_get_band_tuning(net, got), QTN_OK);
  if (got[0].par_bits != 19 || got[1].tile_blocks != 256) ++g_fail;
  qtn_band_tuning bad[QTN_BANDS] = {{40, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  EXPECT(qtn_set_band_tuning(net, bad), QTN_EINVAL);
  const qtn_band_tuning zero[QTN_BANDS] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  EXPECT(qtn_set_band_tuning(net, zero), QTN_OK);
}

static void budgets(qtn_net* net, int m) {
  qtn_info full;
  EXPECT(qtn_get_info(net, &full), QTN_OK);
  // a shared area at half the keep-everything arena, then just below the
  // largest cone's own working set (recomputation)
  const size_t half = full.arena_keep_all / 2;
  if (half > full.pinned_bytes + full.max_cone_dynamic) {
    EXPECT(qtn_set_memory_budget(net, half), QTN_OK);
    check_plan(net, m, true);
  }
  const qtn_status s = qtn_set_memory_budget(net, full.pinned_bytes + full.max_cone_dynamic * 8 / 10);
  if (s != QTN_OK && s != QTN_ENOMEM) {
    std::fprintf(stderr, "budget: status %d (%s)\n", (int)s, qtn_last_error());
    ++g_fail;
  }
  if (s == QTN_OK) check_plan(net, m, true);
  EXPECT(qtn_set_memory_budget(net, 1024), QTN_ENOMEM);
  EXPECT(qtn_set_memory_budget(net, 0), QTN_OK);
  check_plan(net, m, true);
}

static void bad_arguments(qtn_ctx* ctx, int n, const std::vector<int32_t>& edges, int p) {
  qtn_net* net = nullptr;
  const int m = (int)edges.size() / 2;
  EXPECT(qtn_build(nullptr, n, m, edges.data(), p, QTN_C64, &net), QTN_EINVAL);
  EXPECT(qtn_build(ctx, n, m, nullptr, p, QTN_C64, &net), QTN_EINVAL);
  EXPECT(qtn_build(ctx, n, m, edges.data(), 0, QTN_C64, &net), QTN_EINVAL);
  EXPECT(qtn_build(ctx, n, -1, edges.data(), p, QTN_C64, &net), QTN_EINVAL);
  EXPECT(qtn_build(ctx, n, m, edges.data(), p, (qtn_dtype)7, &net), QTN_EINVAL);
  std::vector<int32_t> e2 = edges;
  e2[1] = e2[0];  // self-loop
  EXPECT(qtn_build(ctx, n, m, e2.data(), p, QTN_C64, &net), QTN_EINVAL);
  e2 = edges;
  e2[0] = n;  // vertex out of range
  EXPECT(qtn_build(ctx, n, m, e2.data(), p, QTN_C64, &net), QTN_EINVAL);
  e2 = edges;
  e2[2] = edges[1];
  e2[3] = edges[0];  // the first edge twice
  EXPECT(qtn_build(ctx, n, m, e2.data(), p, QTN_C64, &net), QTN_EINVAL);
  // calls out of order and contractions on a host-only context
  EXPECT(qtn_build(ctx, n, m, edges.data(), p, QTN_C64, &net), QTN_OK);
  size_t ws = 0;
  EXPECT(qtn_validate_plan(net), QTN_ESTATE);
  EXPECT(qtn_workspace_size(net, 1, &ws), QTN_ESTATE);
  std::vector<double> g(p, 0.3), b(p, 0.2);
  EXPECT(qtn_set_params(net, g.data(), b.data()), QTN_ESTATE);
  EXPECT(qtn_order(net, QTN_ORDER_MIN_FILL, nullptr), QTN_OK);
  EXPECT(qtn_set_params(net, nullptr, b.data()), QTN_EINVAL);
  g[0] = std::nan("");
  EXPECT(qtn_set_params(net, g.data(), b.data()), QTN_EINVAL);
  double e = 0;
  EXPECT(qtn_contract(net, QTN_BATCHED, nullptr, 0, nullptr, nullptr, &e), QTN_ESTATE);
  qtn_net_free(net);
  qtn_net_free(nullptr);
}

static void cost_models(int n, const std::vector<int32_t>& edges, int p) {
  const int m = (int)edges.size() / 2;
  for (int v = 0; v < 4; ++v)
    for (int k = 0; k < 2; ++k) {
      qtn_cost c;
      EXPECT(qtn_cost_model(n, m, edges.data(), p, (qtn_net_variant)v, (qtn_order_kind)k, v == 3 ? 2 : 0, 0.5, 7, &c),
             QTN_OK);
      if (c.width < 1 || c.n_indices < 1 || !(c.log2_ops > 0)) {
        std::fprintf(stderr, "cost model variant %d: width %d indices %d log2 %g\n", v, c.width, c.n_indices,
                     c.log2_ops);
        ++g_fail;
      }
    }
  qtn_cost c;
  EXPECT(qtn_cost_model(n, m, edges.data(), p, (qtn_net_variant)9, QTN_ORDER_MIN_FILL, 0, 0.5, 7, &c), QTN_EINVAL);
  // the exported order is a permutation of the indices; a short buffer is refused
  EXPECT(qtn_cost_model(n, m, edges.data(), p, QTN_NET_DIAGONAL_ZZ, QTN_ORDER_MIN_FILL, 2, 0.5, 7, &c), QTN_OK);
  std::vector<int32_t> order(c.n_indices, -1), seen(c.n_indices, 0);
  EXPECT(qtn_cost_model_order(n, m, edges.data(), p, QTN_NET_DIAGONAL_ZZ, QTN_ORDER_MIN_FILL, 2, 0.5, 7, &c,
                              order.data(), (int32_t)order.size()),
         QTN_OK);
  for (int32_t v : order)
    if (v < 0 || v >= c.n_indices || seen[v]++) {
      std::fprintf(stderr, "exported order is not a permutation\n");
      ++g_fail;
      break;
    }
  EXPECT(qtn_cost_model_order(n, m, edges.data(), p, QTN_NET_DIAGONAL_ZZ, QTN_ORDER_MIN_FILL, 2, 0.5, 7, &c,
                              order.data(), (int32_t)order.size() - 1),
         QTN_EINVAL);
}

int main(int argc, char** argv) {
  if (argc != 2) {
    std::fprintf(stderr, "usage: %s graphs.txt\n", argv[0]);
    return 2;
  }
  qtn_ctx* ctx = nullptr;
  EXPECT(qtn_create(QTN_HOST_ONLY, &ctx), QTN_OK);
  if (!ctx) return 1;
  std::ifstream in(argv[1]);
  std::string line;
  int cases = 0;
  while (std::getline(in, line)) {
    if (line.empty() || line[0] == '#') continue;
    std::istringstream ss(line);
    std::string kind;
    int n, p, m;
    ss >> kind >> n >> p >> m;
    std::vector<int32_t> edges(2 * m);
    for (auto& x : edges) ss >> x;
    const bool amp = kind == "amp";
    for (int dt = 0; dt < (kind == "qaoa64" ? 1 : 2); ++dt) {
      qtn_net* net = nullptr;
      if (amp)
        EXPECT(qtn_build_amplitude(ctx, n, m, edges.data(), p, (qtn_dtype)dt, &net), QTN_OK);
      else
        EXPECT(qtn_build(ctx, n, m, edges.data(), p, (qtn_dtype)dt, &net), QTN_OK);
      if (!net) continue;
      int32_t w1 = 0, w2 = 0;
      EXPECT(qtn_order(net, QTN_ORDER_MIN_FILL, &w1), QTN_OK);
      check_plan(net, m, !amp);
      EXPECT(qtn_order_rgreedy(net, QTN_ORDER_MIN_DEGREE, 3, 0.5, 11, &w2), QTN_OK);
      check_plan(net, m, !amp);
      if (w1 < 1 || w2 < 1) ++g_fail;
      tunings(net, m, !amp);
      if (!amp) budgets(net, m);
      qtn_net_free(net);
    }
    if (!amp) {
      bad_arguments(ctx, n, edges, p);
      if (n <= 16) cost_models(n, edges, p);
    }
    ++cases;
  }
  qtn_destroy(ctx);
  std::printf("%d graphs, %d unexpected results\n", cases, g_fail);
  return g_fail ? 1 : 0;
}
