// C ABI of the library (declared in include/qtn.h).  Host orchestration:
// plan upload, leaf values, plain per-op launches, the persistent sweep and
// its hipGraph, result read-back, autotuning.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdint>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <exception>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "../../include/qtn.h"
#include "kernels.hpp"
#include "plan.hpp"

static_assert(qtn::kScratchBytes == QTN_SCRATCH_BYTES, "scratch size of the header and the kernels differ");

using namespace qtn;

namespace {
thread_local std::string g_err;

qtn_status fail(qtn_status s, const std::string& msg) {
  g_err = msg;
  return s;
}
#define HIPCHECK(call)                                                                              \
  do {                                                                                              \
    hipError_t e_ = (call);                                                                         \
    if (e_ != hipSuccess) return fail(QTN_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

size_t align256(size_t x) { return (x + 255) / 256 * 256; }
// Upper bound on the polls of one dependency wait in the persistent kernel
// (~1 us each): a plan bug makes the sweep report an error instead of hanging.
constexpr long long kSpinLimit = 20000000LL;
}  // namespace

struct qtn_ctx {
  int device = 0;
  int n_cu = 256;
  hipStream_t cap_stream = nullptr;
  void* scratch = nullptr;  // device address of this device's static scratch (allocation-free entry point)
};

struct DevProg {
  QItem* items = nullptr;
  int32_t* succ = nullptr;
  int32_t* init = nullptr;
  int32_t* small_items = nullptr;  // (lo, hi) per LDS-resident cone
  int32_t n_items = 0, n_nodes = 0, n_small = 0;
};

struct GraphCache {
  hipGraphExec_t exec = nullptr;
  void* ws = nullptr;
  void* zz = nullptr;
  bool valid = false;
};

struct qtn_net {
  qtn_ctx* ctx = nullptr;
  Plan P;
  bool c128 = false;
  int elem = 8;
  // device plan
  OpDesc* d_ops = nullptr;
  LeafRef* d_leafrefs = nullptr;
  SmallOp* d_small = nullptr;  // LDS-resident programs
  DevProg prog[2];
  void* d_leafvals = nullptr;  // vals then dvals, element type
  // host staging (pinned)
  void* h_leafvals = nullptr;
  double* h_fin = nullptr;
  void* dh_leafvals = nullptr;  // device addresses of the two mapped pinned host buffers
  void* dh_fin = nullptr;
  size_t leaf_bytes = 0;
  bool params_set = false;
  int grid = 0;
  int max_nin = 1;
  bool has_wide = false;  // some op carries F_WIDE
  bool amplitude = false; // single-amplitude network (one cone, result = <0...0|gamma beta>)
  GraphCache graph[2];
  hipEvent_t ev_k0 = nullptr, ev_k1 = nullptr, ev_done = nullptr;
  bool ev_pending = false;
  bool sweep_timing = false;  // HIP events around each batched graph replay (qtn_set_sweep_timing)
  double kernel_ms_sum = 0;
  int64_t kernel_count = 0;
  std::vector<double> gamma, beta;
  // the last sweep enqueued: its mode (-1: none yet), whether it ran the
  // adjoint, and its workspace (qtn_edge_results reads it)
  int last_mode = -1;
  bool last_grad = false;
  const void* last_ws = nullptr;
};

namespace {

// Workspace layout: [res: n_cones*(2+4p) doubles][fin: 1+2p doubles][ctl: 2+n_nodes int32][arena]
struct WsLayout {
  size_t res_off, fin_off, ctl_off, arena_off, total;
};

WsLayout ws_layout(const qtn_net* n, bool grad) {
  WsLayout L;
  const size_t nc = n->P.cones.size();
  const int rs = 2 + 4 * n->P.p;
  L.res_off = 0;
  L.fin_off = align256(nc * rs * sizeof(double));
  L.ctl_off = L.fin_off + align256((1 + 2 * n->P.p) * sizeof(double));
  const int nn = std::max(n->prog[0].n_nodes, n->prog[1].n_nodes);
  L.arena_off = L.ctl_off + align256((2 + nn) * sizeof(int32_t));
  L.total = L.arena_off + align256((size_t)(grad ? n->P.arena_grad : n->P.arena_fwd) * n->elem);
  return L;
}

// Bytes copied back after every sweep: the fin block (E, dE/dgamma,
// dE/dbeta) through the queue head and error flag of the ctl block.
size_t fin_copy_bytes(const qtn_net* n) {
  const WsLayout L = ws_layout(n, true);
  return (L.ctl_off - L.fin_off) + 2 * sizeof(int32_t);
}

void free_device_plan(qtn_net* n) {
  (void)hipFree(n->d_ops);
  (void)hipFree(n->d_leafrefs);
  (void)hipFree(n->d_small);
  n->d_small = nullptr;
  for (auto& pg : n->prog) {
    (void)hipFree(pg.items);
    (void)hipFree(pg.succ);
    (void)hipFree(pg.init);
    (void)hipFree(pg.small_items);
    pg = DevProg();
  }
  n->d_ops = nullptr;
  n->d_leafrefs = nullptr;
  for (auto& g : n->graph) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    g = GraphCache();
  }
}

template <typename T>
hipError_t upload(T** dst, const std::vector<T>& src) {
  size_t bytes = std::max<size_t>(sizeof(T), src.size() * sizeof(T));
  hipError_t e = hipMalloc((void**)dst, bytes);
  if (e != hipSuccess) return e;
  if (!src.empty()) e = hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice);
  return e;
}

qtn_status rebuild_programs(qtn_net* n) {
  // workgroups resident at once: 16 wavefronts per compute unit (the
  // persistent kernel's register budget), at most the launched grid
  const int waves_per_wg = std::max(1, n->P.tune.threads / 64);
  n->P.sched_workers = std::max(1, std::min(n->grid, n->ctx->n_cu * std::max(1, 16 / waves_per_wg)));
  std::string err = build_programs(n->P, n->elem);
  if (!err.empty()) return fail(QTN_EUNSUPPORTED, err);
  build_items(n->P, false);
  build_items(n->P, true);
  n->max_nin = 1;
  for (const OpDesc& d : n->P.ops)
    if (d.kind == OP_CONTRACT || d.kind == OP_ADJOINT) n->max_nin = std::max(n->max_nin, (int)d.n_in);
  n->has_wide = false;
  for (const OpDesc& d : n->P.ops)
    n->has_wide |= (d.kind == OP_CONTRACT && (d.flags & F_WIDE)) || d.kind == OP_ADJOINT;
  if (n->ctx->device < 0) {  // host-only context: plan without upload
    for (int g = 0; g < 2; ++g)
      n->prog[g].n_nodes = (int32_t)(g ? n->P.node_init_grad.size() : n->P.node_init_fwd.size());
    return QTN_OK;
  }
  HIPCHECK(hipSetDevice(n->ctx->device));
  free_device_plan(n);
  HIPCHECK(upload(&n->d_ops, n->P.ops));
  HIPCHECK(upload(&n->d_leafrefs, n->P.leafrefs));
  HIPCHECK(upload(&n->d_small, n->P.small));
  for (int g = 0; g < 2; ++g) {
    DevProg& pg = n->prog[g];
    const auto& items = g ? n->P.items_grad : n->P.items_fwd;
    const auto& succ = g ? n->P.succ_grad : n->P.succ_fwd;
    const auto& init = g ? n->P.node_init_grad : n->P.node_init_fwd;
    const auto& small_items = g ? n->P.small_items_grad : n->P.small_items_fwd;
    HIPCHECK(upload(&pg.items, items));
    HIPCHECK(upload(&pg.succ, succ));
    HIPCHECK(upload(&pg.init, init));
    HIPCHECK(upload(&pg.small_items, small_items));
    pg.n_items = (int32_t)items.size();
    pg.n_nodes = (int32_t)init.size();
    pg.n_small = (int32_t)(small_items.size() / 2);
  }
  return QTN_OK;
}

Env make_env(qtn_net* n, char* ws, const WsLayout& L) {
  Env e;
  e.arena = ws + L.arena_off;
  e.res = reinterpret_cast<double*>(ws + L.res_off);
  e.leafvals = n->d_leafvals;
  e.dleafvals = (char*)n->d_leafvals + n->leaf_bytes / 2;
  e.leafrefs = n->d_leafrefs;
  e.p = n->P.p;
  e.res_stride = 2 + 4 * n->P.p;
  return e;
}

// Enqueue one complete sweep on stream st (no host synchronisation).  With
// pk0/pk1 (not under capture) the persistent kernel is bracketed by them.
qtn_status enqueue_sweep(qtn_net* n, int mode, bool grad, void* ws, hipStream_t st, void* zz_out,
                         hipEvent_t pk0 = nullptr, hipEvent_t pk1 = nullptr) {
  n->last_mode = mode;
  n->last_grad = grad;
  n->last_ws = ws;
  const WsLayout L = ws_layout(n, grad);
  char* w = static_cast<char*>(ws);
  Env env = make_env(n, w, L);
  // kernel launches report through hipGetLastError: drop any error left
  // behind by unrelated earlier calls on this thread
  (void)hipGetLastError();
  const TuneParams& T = n->P.tune;
  DevProg& pg = n->prog[grad ? 1 : 0];
  int32_t* ctl = reinterpret_cast<int32_t*>(w + L.ctl_off);
  const bool batched = mode == QTN_BATCHED;
  // leaf-product tables; the batched form also resets the queue, in the leaf
  // launch or, without one, in the copy of the leaf values
  const int32_t leaf_hi = n->P.leaf_hi;
  const int32_t lgrad_hi = n->P.lgrad_hi;
  const bool leaf_launch = leaf_hi > n->P.leaf_lo;
  HIPCHECK(launch_small_copy(n->dh_leafvals, n->d_leafvals, n->leaf_bytes, st,
                             batched && !leaf_launch ? ctl : nullptr, pg.init, pg.n_nodes));
  if (leaf_launch)
    HIPCHECK(launch_batch(n->c128, false, 64, n->d_ops, n->P.leaf_lo, leaf_hi, env, st, batched ? ctl : nullptr, pg.init,
                          pg.n_nodes));
  if (mode == QTN_PLAIN) {
    for (size_t c = 0; c < n->P.cones.size(); ++c) {
      auto run = [&](int32_t lo, int32_t hi) -> qtn_status {
        for (int32_t o = lo; o < hi; ++o) {
          hipError_t e = launch_op(n->c128, n->d_ops, n->P.ops[o], o, env, T.threads, 4096, st);
          if (e != hipSuccess) return fail(QTN_EDEVICE, std::string("op launch: ") + hipGetErrorString(e));
        }
        return QTN_OK;
      };
      qtn_status s;
      if (grad) {
        if ((s = run(n->P.cone_fwd_lo[c], n->P.cone_fwd_hi[c])) != QTN_OK) return s;
        if ((s = run(n->P.cone_adj_lo[c], n->P.cone_adj_hi[c])) != QTN_OK) return s;
      } else {
        if ((s = run(n->P.cone_fwd_lo[c], n->P.cone_fwd_hi[c] + 1)) != QTN_OK) return s;
      }
    }
  } else {
    // the LDS-resident cones (one workgroup each), then the work queue of
    // the others; the two are independent
    const int grid = std::max(1, std::min<int>(n->grid, std::max(1, pg.n_items)));
    const size_t lds_bytes = (size_t)n->P.lds_elems * n->elem;
    if (pk0) HIPCHECK(hipEventRecord(pk0, st));
    HIPCHECK(launch_small(n->c128, n->d_small, pg.small_items, pg.n_small, env, T.lds_threads, lds_bytes, st));
    if (pg.n_items > 0)
      HIPCHECK(launch_persistent(n->c128, n->has_wide, n->max_nin, n->d_ops, pg.items, pg.n_items, pg.succ, ctl, env,
                                 T.threads, grid, lds_bytes, kSpinLimit, st));
    if (pk1) HIPCHECK(hipEventRecord(pk1, st));
  }
  if (grad && n->P.lgrad_mid > n->P.lgrad_lo)
    HIPCHECK(launch_batch(n->c128, true, 8, n->d_ops, n->P.lgrad_lo, n->P.lgrad_mid, env, st));
  if (grad && lgrad_hi > n->P.lgrad_mid)
    HIPCHECK(launch_batch(n->c128, true, 64, n->d_ops, n->P.lgrad_mid, lgrad_hi, env, st));
  // E, dE/dtheta straight into the mapped host buffer, followed (at the
  // workspace's ctl offset) by the queue head and the persistent kernel's
  // error flag
  HIPCHECK(launch_final(n->c128, env.res, env.res_stride, (int)n->P.cones.size(), n->P.p, grad ? 1 : 0, zz_out,
                        reinterpret_cast<double*>(w + L.fin_off), static_cast<double*>(n->dh_fin),
                        mode == QTN_BATCHED ? ctl : nullptr,
                        reinterpret_cast<int32_t*>(static_cast<char*>(n->dh_fin) + (L.ctl_off - L.fin_off)), st));
  return QTN_OK;
}

// Waits for the last sweep's completion event.  Polls rather than blocks: a
// blocking wait can add a scheduler wake-up (up to a millisecond) to every
// sweep.
hipError_t wait_done(qtn_net* n) {
  hipError_t q;
  while ((q = hipEventQuery(n->ev_done)) == hipErrorNotReady) std::this_thread::yield();
  return q;
}

// The persistent kernel's error flag as the final kernel copied it into the
// mapped host buffer (valid once the sweep has completed).
int32_t sweep_flag(const qtn_net* n) {
  const WsLayout L = ws_layout(n, true);
  int32_t flag = 0;
  std::memcpy(&flag, reinterpret_cast<const char*>(n->h_fin) + (L.ctl_off - L.fin_off) + sizeof(int32_t),
              sizeof(int32_t));
  return flag;
}

qtn_status check_ready(qtn_net* n, void* ws, size_t ws_bytes, bool grad) {
  if (!n) return fail(QTN_EINVAL, "net is NULL");
  if (n->ctx->device < 0) return fail(QTN_ESTATE, "host-only context cannot run contractions");
  if (!n->P.ordered || !n->d_ops) return fail(QTN_ESTATE, "qtn_order has not been called");
  if (!n->params_set) return fail(QTN_ESTATE, "qtn_set_params has not been called");
  const WsLayout L = ws_layout(n, grad);
  if (!ws && L.total) return fail(QTN_EINVAL, "workspace is NULL");
  if ((uintptr_t)ws % 256) return fail(QTN_EINVAL, "workspace must be 256-byte aligned");
  if (ws_bytes < L.total)
    return fail(QTN_ENOMEM, "workspace has " + std::to_string(ws_bytes) + " bytes, needs " + std::to_string(L.total));
  return QTN_OK;
}

qtn_status run_sweep(qtn_net* n, int mode, bool grad, void* ws, size_t ws_bytes, hipStream_t st, void* zz_out,
                     bool want_host) {
  HIPCHECK(hipSetDevice(n->ctx->device));
  if (mode == QTN_BATCHED) {
    GraphCache& g = n->graph[grad ? 1 : 0];
    // the workspace and zz_out pointers are baked into the graph: re-capture
    // when either changes
    const bool reuse = g.valid && g.ws == ws && g.zz == zz_out;
    if (!reuse) {
      if (g.exec) (void)hipGraphExecDestroy(g.exec);
      g = GraphCache();
      hipStream_t cs = n->ctx->cap_stream;
      HIPCHECK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
      qtn_status s = enqueue_sweep(n, mode, grad, ws, cs, zz_out);
      hipGraph_t graph = nullptr;
      hipError_t e = hipStreamEndCapture(cs, &graph);
      if (s != QTN_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return s;
      }
      if (e != hipSuccess) return fail(QTN_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
      e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (e != hipSuccess) return fail(QTN_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
      g.ws = ws;
      g.zz = zz_out;
      g.valid = true;
    }
    // events on the caller's stream around the replay time the device work
    // of the whole sweep (events recorded inside a captured graph carry no
    // timestamps)
    n->last_mode = mode;
    n->last_grad = grad;
    n->last_ws = ws;
    if (n->sweep_timing) {
      HIPCHECK(hipEventRecord(n->ev_k0, st));
      HIPCHECK(hipGraphLaunch(g.exec, st));
      HIPCHECK(hipEventRecord(n->ev_k1, st));
      n->ev_pending = true;
    } else {
      HIPCHECK(hipGraphLaunch(g.exec, st));
    }
  } else {
    qtn_status s = enqueue_sweep(n, mode, grad, ws, st, zz_out);
    if (s != QTN_OK) return s;
  }
  HIPCHECK(hipEventRecord(n->ev_done, st));
  if (want_host) {
    hipError_t q = wait_done(n);
    if (q != hipSuccess) return fail(QTN_EDEVICE, std::string("sweep: ") + hipGetErrorString(q));
    if (mode == QTN_BATCHED && n->ev_pending) {
      float ms = 0;
      if (hipEventElapsedTime(&ms, n->ev_k0, n->ev_k1) == hipSuccess) {
        n->kernel_ms_sum += ms;
        n->kernel_count += 1;
      } else {
        (void)hipGetLastError();
      }
      n->ev_pending = false;
    }
    if (mode == QTN_BATCHED && sweep_flag(n)) return fail(QTN_EDEVICE, "persistent sweep gave up waiting on a dependency");
  }
  return QTN_OK;
}

}  // namespace

extern "C" {

const char* qtn_last_error(void) { return g_err.c_str(); }

qtn_status qtn_create(int device, qtn_ctx** out) {
  if (!out) return fail(QTN_EINVAL, "out is NULL");
  *out = nullptr;
  if (device == QTN_HOST_ONLY) {
    qtn_ctx* c = new (std::nothrow) qtn_ctx();
    if (!c) return fail(QTN_ENOMEM, "host allocation failed");
    c->device = QTN_HOST_ONLY;
    *out = c;
    return QTN_OK;
  }
  int ndev = 0;
  HIPCHECK(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fail(QTN_EINVAL, "device id out of range");
  HIPCHECK(hipSetDevice(device));
  qtn_ctx* c = new (std::nothrow) qtn_ctx();
  if (!c) return fail(QTN_ENOMEM, "host allocation failed");
  c->device = device;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) c->n_cu = prop.multiProcessorCount;
  if (hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) {
    delete c;
    return fail(QTN_EDEVICE, "stream creation failed");
  }
  // the static scratch's device address on this device (current here)
  hipError_t se = scratch_address(device, &c->scratch);
  if (se != hipSuccess || !c->scratch) {
    (void)hipStreamDestroy(c->cap_stream);
    delete c;
    return fail(QTN_EDEVICE, std::string("static scratch address: ") + hipGetErrorString(se));
  }
  *out = c;
  return QTN_OK;
}

void qtn_destroy(qtn_ctx* c) {
  if (!c) return;
  if (c->device < 0) {
    delete c;
    return;
  }
  (void)hipSetDevice(c->device);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  delete c;
}

static qtn_status build_net(qtn_ctx* ctx, int32_t n_vertices, int32_t n_edges, const int32_t* edges, int32_t p,
                            qtn_dtype dtype, bool amplitude, qtn_net** out) {
  if (!ctx || !out) return fail(QTN_EINVAL, "ctx or out is NULL");
  *out = nullptr;
  if (dtype != QTN_C64 && dtype != QTN_C128) return fail(QTN_EINVAL, "unknown dtype");
  std::string err = validate_graph(n_vertices, n_edges, edges, p);
  if (!err.empty()) return fail(QTN_EINVAL, err);
  try {
    qtn_net* n = new qtn_net();
    n->ctx = ctx;
    n->c128 = dtype == QTN_C128;
    n->elem = n->c128 ? 16 : 8;
    n->P.n = n_vertices;
    n->P.p = p;
    for (int e = 0; e < n_edges; ++e) n->P.edges.push_back({edges[2 * e], edges[2 * e + 1]});
    n->amplitude = amplitude;
    if (amplitude)
      build_amplitude(n->P);
    else
      build_cones(n->P);
    n->grid = 8 * ctx->n_cu;
    *out = n;
    return QTN_OK;
  } catch (const std::bad_alloc&) {
    return fail(QTN_ENOMEM, "host allocation failed");
  } catch (const std::exception& ex) {
    return fail(QTN_EINVAL, ex.what());
  }
}

qtn_status qtn_build(qtn_ctx* ctx, int32_t n_vertices, int32_t n_edges, const int32_t* edges, int32_t p,
                     qtn_dtype dtype, qtn_net** out) {
  return build_net(ctx, n_vertices, n_edges, edges, p, dtype, false, out);
}

qtn_status qtn_build_amplitude(qtn_ctx* ctx, int32_t n_vertices, int32_t n_edges, const int32_t* edges, int32_t p,
                               qtn_dtype dtype, qtn_net** out) {
  if (n_vertices < 1) return fail(QTN_EINVAL, "the amplitude network needs at least one vertex");
  return build_net(ctx, n_vertices, n_edges, edges, p, dtype, true, out);
}

qtn_status qtn_amplitude(qtn_net* n, qtn_mode mode, void* ws, size_t ws_bytes, void* stream, double* amp_out,
                         double* damp_out) {
  if (mode != QTN_PLAIN && mode != QTN_BATCHED) return fail(QTN_EINVAL, "unknown mode");
  if (!n || !amp_out) return fail(QTN_EINVAL, "net or amp_out is NULL");
  if (!n->amplitude) return fail(QTN_ESTATE, "not an amplitude network (use qtn_build_amplitude)");
  const bool grad = damp_out != nullptr;
  qtn_status s = check_ready(n, ws, ws_bytes, grad);
  if (s != QTN_OK) return s;
  s = run_sweep(n, mode, grad, ws, ws_bytes, (hipStream_t)stream, nullptr, true);
  if (s != QTN_OK) return s;
  const int rs = 2 + 4 * n->P.p;
  std::vector<double> r(rs);
  HIPCHECK(hipMemcpy(r.data(), ws, rs * sizeof(double), hipMemcpyDeviceToHost));  // the one cone's record
  amp_out[0] = r[0];
  amp_out[1] = r[1];
  if (grad)
    for (int i = 0; i < 4 * n->P.p; ++i) damp_out[i] = r[2 + i];
  return QTN_OK;
}

qtn_status qtn_order(qtn_net* n, qtn_order_kind kind, int32_t* max_width_out) {
  return qtn_order_rgreedy(n, kind, 0, 0.0, 0, max_width_out);
}

qtn_status qtn_order_rgreedy(qtn_net* n, qtn_order_kind kind, int32_t n_repeats, double temperature, uint64_t seed,
                             int32_t* max_width_out) {
  if (!n) return fail(QTN_EINVAL, "net is NULL");
  if (kind != QTN_ORDER_MIN_DEGREE && kind != QTN_ORDER_MIN_FILL) return fail(QTN_EINVAL, "unknown order kind");
  if (n_repeats < 0 || !(temperature >= 0.0) || !std::isfinite(temperature))
    return fail(QTN_EINVAL, "n_repeats must be >= 0 and temperature finite and >= 0");
  try {
    unsigned hw = std::thread::hardware_concurrency();
    OrderOptions O;
    O.kind = (int)kind;
    O.repeats = n_repeats;
    O.temperature = temperature;
    O.seed = seed;
    order_cones(n->P, O, (int)std::max(1u, std::min(hw, 16u)));
    if (n->P.max_width > MAXBITS - 1)
      return fail(QTN_EUNSUPPORTED, "contraction width " + std::to_string(n->P.max_width) + " exceeds 30");
    qtn_status s = rebuild_programs(n);
    if (s != QTN_OK) return s;
    n->leaf_bytes = 2 * (size_t)n_leaf_kinds(n->P.p) * 4 * n->elem;
    if (n->ctx->device < 0) {
      if (!n->h_leafvals) n->h_leafvals = std::calloc(1, n->leaf_bytes);
      if (!n->h_leafvals) return fail(QTN_ENOMEM, "host allocation failed");
      if (max_width_out) *max_width_out = n->P.max_width;
      return QTN_OK;
    }
    HIPCHECK(hipSetDevice(n->ctx->device));
    if (!n->d_leafvals) {
      n->leaf_bytes = 2 * (size_t)n_leaf_kinds(n->P.p) * 4 * n->elem;
      HIPCHECK(hipMalloc(&n->d_leafvals, n->leaf_bytes));
      HIPCHECK(hipHostMalloc(&n->h_leafvals, n->leaf_bytes, hipHostMallocMapped));
      HIPCHECK(hipHostMalloc((void**)&n->h_fin, fin_copy_bytes(n), hipHostMallocMapped));
      HIPCHECK(hipHostGetDevicePointer(&n->dh_leafvals, n->h_leafvals, 0));
      HIPCHECK(hipHostGetDevicePointer(&n->dh_fin, n->h_fin, 0));
      HIPCHECK(hipEventCreate(&n->ev_k0));
      HIPCHECK(hipEventCreate(&n->ev_k1));
      HIPCHECK(hipEventCreateWithFlags(&n->ev_done, hipEventDisableTiming));
      std::memset(n->h_leafvals, 0, n->leaf_bytes);
    }
    if (max_width_out) *max_width_out = n->P.max_width;
    return QTN_OK;
  } catch (const std::bad_alloc&) {
    return fail(QTN_ENOMEM, "host allocation failed");
  }
}

qtn_status qtn_workspace_size(const qtn_net* n, int32_t with_grad, size_t* bytes_out) {
  if (!n || !bytes_out) return fail(QTN_EINVAL, "net or bytes_out is NULL");
  if (!n->P.ordered) return fail(QTN_ESTATE, "qtn_order has not been called");
  *bytes_out = ws_layout(n, with_grad != 0).total;
  return QTN_OK;
}

qtn_status qtn_set_params(qtn_net* n, const double* gamma, const double* beta) {
  if (!n) return fail(QTN_EINVAL, "net is NULL");
  if (!n->h_leafvals) return fail(QTN_ESTATE, "qtn_order has not been called");
  const int p = n->P.p;
  if (p > 0 && (!gamma || !beta)) return fail(QTN_EINVAL, "gamma or beta is NULL");
  for (int l = 0; l < p; ++l)
    if (!std::isfinite(gamma[l]) || !std::isfinite(beta[l])) return fail(QTN_EINVAL, "non-finite angle");
  // the previous sweep may still read the staging buffer
  if (n->ev_done) HIPCHECK(hipEventSynchronize(n->ev_done));
  if (!n->h_leafvals) return fail(QTN_ESTATE, "qtn_order has not been called");
  const int nk = n_leaf_kinds(p);
  std::vector<double> v((size_t)nk * 8, 0.0), dv((size_t)nk * 8, 0.0);  // [kind][entry][re,im]
  auto put = [&](std::vector<double>& a, int kind, int e, double re, double im) {
    a[((size_t)kind * 4 + e) * 2] = re;
    a[((size_t)kind * 4 + e) * 2 + 1] = im;
  };
  const double h = std::sqrt(0.5);
  put(v, LK_PLUS, 0, h, 0);
  put(v, LK_PLUS, 1, h, 0);
  put(v, LK_ZOBS, 0, 1, 0);
  put(v, LK_ZOBS, 1, -1, 0);
  put(v, lk_proj0(p), 0, 1, 0);  // <0|: entry 1 stays 0
  for (int l = 0; l < p; ++l) {
    // ZZ phase of exp(-i gamma C) on one edge: 1 if the bits agree, exp(-i gamma) if not
    const double cg = std::cos(gamma[l]), sg = std::sin(gamma[l]);
    const double cb = std::cos(beta[l]), sb = std::sin(beta[l]);
    for (int conj = 0; conj < 2; ++conj) {
      const double sgn = conj ? -1.0 : 1.0;
      const int kz = conj ? lk_zzb(l) : lk_zz(l);
      put(v, kz, 0, 1, 0);
      put(v, kz, 3, 1, 0);
      put(v, kz, 1, cg, -sgn * sg);
      put(v, kz, 2, cg, -sgn * sg);
      // d/dgamma exp(-i s gamma) = -i s exp(-i s gamma)
      put(dv, kz, 1, -sg, -sgn * cg);
      put(dv, kz, 2, -sg, -sgn * cg);
      // mixer exp(-i beta X) = [[cos, -i sin], [-i sin, cos]] (conjugated on the bra)
      const int km = conj ? lk_mxb(l) : lk_mx(l);
      put(v, km, 0, cb, 0);
      put(v, km, 3, cb, 0);
      put(v, km, 1, 0, -sgn * sb);
      put(v, km, 2, 0, -sgn * sb);
      put(dv, km, 0, -sb, 0);
      put(dv, km, 3, -sb, 0);
      put(dv, km, 1, 0, -sgn * cb);
      put(dv, km, 2, 0, -sgn * cb);
    }
  }
  const size_t half = n->leaf_bytes / 2;
  if (n->c128) {
    std::memcpy(n->h_leafvals, v.data(), half);
    std::memcpy((char*)n->h_leafvals + half, dv.data(), half);
  } else {
    float* f = static_cast<float*>(n->h_leafvals);
    for (size_t i = 0; i < v.size(); ++i) f[i] = (float)v[i];
    for (size_t i = 0; i < dv.size(); ++i) f[v.size() + i] = (float)dv[i];
  }
  n->gamma.assign(gamma, gamma + p);
  n->beta.assign(beta, beta + p);
  n->params_set = true;
  return QTN_OK;
}

qtn_status qtn_contract(qtn_net* n, qtn_mode mode, void* ws, size_t ws_bytes, void* stream, void* zz_out,
                        double* energy_out) {
  if (mode != QTN_PLAIN && mode != QTN_BATCHED) return fail(QTN_EINVAL, "unknown mode");
  qtn_status s = check_ready(n, ws, ws_bytes, false);
  if (s != QTN_OK) return s;
  s = run_sweep(n, mode, false, ws, ws_bytes, (hipStream_t)stream, zz_out, energy_out != nullptr);
  if (s != QTN_OK) return s;
  if (energy_out) *energy_out = n->h_fin[0];
  return QTN_OK;
}

qtn_status qtn_energy_grad(qtn_net* n, qtn_mode mode, void* ws, size_t ws_bytes, void* stream, void* zz_out,
                           double* energy_out, double* dgamma_out, double* dbeta_out) {
  if (mode != QTN_PLAIN && mode != QTN_BATCHED) return fail(QTN_EINVAL, "unknown mode");
  if (!energy_out) return fail(QTN_EINVAL, "energy_out is NULL");
  if ((dgamma_out == nullptr) != (dbeta_out == nullptr)) return fail(QTN_EINVAL, "dgamma_out/dbeta_out mismatch");
  qtn_status s = check_ready(n, ws, ws_bytes, true);
  if (s != QTN_OK) return s;
  s = run_sweep(n, mode, true, ws, ws_bytes, (hipStream_t)stream, zz_out, true);
  if (s != QTN_OK) return s;
  const int p = n->P.p;
  *energy_out = n->h_fin[0];
  if (dgamma_out)
    for (int l = 0; l < p; ++l) {
      dgamma_out[l] = n->h_fin[1 + l];
      dbeta_out[l] = n->h_fin[1 + p + l];
    }
  return QTN_OK;
}

qtn_status qtn_energy_grad_noalloc(qtn_net* n, qtn_mode mode, void* stream, void* zz_out, double* energy_out,
                                   double* dgamma_out, double* dbeta_out) {
  if (mode != QTN_PLAIN && mode != QTN_BATCHED) return fail(QTN_EINVAL, "unknown mode");
  if (!n) return fail(QTN_EINVAL, "net is NULL");
  if (!energy_out) return fail(QTN_EINVAL, "energy_out is NULL");
  if ((dgamma_out == nullptr) != (dbeta_out == nullptr)) return fail(QTN_EINVAL, "dgamma_out/dbeta_out mismatch");
  if (n->ctx->device < 0) return fail(QTN_ESTATE, "host-only context cannot run contractions");
  if (!n->P.ordered || !n->d_ops) return fail(QTN_ESTATE, "qtn_order has not been called");
  void* ws = n->ctx->scratch;
  if (!ws) return fail(QTN_EDEVICE, "the static scratch has no device address");
  const size_t need = ws_layout(n, true).total;
  if (need > kScratchBytes)
    return fail(QTN_ENOMEM, "the network needs " + std::to_string(need) + " bytes of workspace; the static scratch " +
                                "of the allocation-free entry point holds " + std::to_string(kScratchBytes));
  qtn_status s = check_ready(n, ws, kScratchBytes, true);
  if (s != QTN_OK) return s;
  HIPCHECK(hipSetDevice(n->ctx->device));
  hipStream_t st = (hipStream_t)stream;
  // kernels launched directly on the caller's stream: no graph capture or
  // instantiation, nothing allocated
  s = enqueue_sweep(n, mode, true, ws, st, zz_out);
  if (s != QTN_OK) return s;
  HIPCHECK(hipEventRecord(n->ev_done, st));
  hipError_t q = wait_done(n);
  if (q != hipSuccess) return fail(QTN_EDEVICE, std::string("sweep: ") + hipGetErrorString(q));
  if (mode == QTN_BATCHED && sweep_flag(n)) return fail(QTN_EDEVICE, "persistent sweep gave up waiting on a dependency");
  const int p = n->P.p;
  *energy_out = n->h_fin[0];
  if (dgamma_out)
    for (int l = 0; l < p; ++l) {
      dgamma_out[l] = n->h_fin[1 + l];
      dbeta_out[l] = n->h_fin[1 + p + l];
    }
  return QTN_OK;
}

qtn_status qtn_edge_results(qtn_net* n, const void* ws, void* stream, double* zz, double* dzz) {
  if (!n) return fail(QTN_EINVAL, "net is NULL");
  if (n->ctx->device < 0) return fail(QTN_ESTATE, "host-only context has no device results");
  if (!n->P.ordered) return fail(QTN_ESTATE, "qtn_order has not been called");
  if (n->last_mode < 0) return fail(QTN_ESTATE, "no sweep has run");
  if (!ws) ws = n->last_ws;
  if (ws != n->last_ws) return fail(QTN_EINVAL, "workspace is not the one the last sweep used");
  if (dzz && !n->last_grad) return fail(QTN_ESTATE, "the last sweep computed no gradient");
  HIPCHECK(hipSetDevice(n->ctx->device));
  HIPCHECK(hipStreamSynchronize((hipStream_t)stream));
  HIPCHECK(hipEventSynchronize(n->ev_done));
  if (n->last_mode == QTN_BATCHED && sweep_flag(n))
    return fail(QTN_EDEVICE, "persistent sweep gave up waiting on a dependency");
  const size_t nc = n->P.cones.size();
  const int rs = 2 + 4 * n->P.p;
  std::vector<double> res(nc * rs);
  if (nc) HIPCHECK(hipMemcpy(res.data(), ws, res.size() * sizeof(double), hipMemcpyDeviceToHost));
  for (size_t c = 0; c < nc; ++c) {
    if (zz) {
      zz[2 * c] = res[c * rs];
      zz[2 * c + 1] = res[c * rs + 1];
    }
    if (dzz)
      for (int t = 0; t < 4 * n->P.p; ++t) dzz[c * 4 * n->P.p + t] = res[c * rs + 2 + t];
  }
  return QTN_OK;
}

qtn_status qtn_gemm_census(const qtn_net* n, int32_t min_bits, int64_t* n_steps, int64_t* n_gemm, double* gemm_flops,
                           double* total_flops) {
  if (!n) return fail(QTN_EINVAL, "net is NULL");
  if (!n->P.ordered) return fail(QTN_ESTATE, "qtn_order has not been called");
  if (min_bits < 1) return fail(QTN_EINVAL, "min_bits must be >= 1");
  int64_t steps = 0, gemm = 0;
  double fg = 0, ft = 0;
  for (const Cone& C : n->P.cones)
    for (const Bucket& B : C.buckets) {
      std::vector<uint32_t> in(B.in_mask.begin(), B.in_mask.end());
      if (B.lam_mask) in.push_back(B.lam_mask);
      const uint32_t summed = B.elim_mask();
      const double f = 6.0 * std::max<int>((int)in.size() - 1, 0) * std::ldexp(1.0, B.nbits()) +
                       2.0 * std::ldexp(1.0, B.nbits());
      bool dense = false;
      for (size_t a = 0; a < in.size() && !dense; ++a)
        for (size_t b = a + 1; b < in.size() && !dense; ++b) {
          const int k = __builtin_popcount(in[a] & in[b] & summed);
          const int m = __builtin_popcount(in[a] & ~in[b] & ~summed);
          const int nn = __builtin_popcount(in[b] & ~in[a] & ~summed);
          dense = k >= min_bits && m >= min_bits && nn >= min_bits;
        }
      ++steps;
      ft += f;
      if (dense) {
        ++gemm;
        fg += f;
      }
    }
  if (n_steps) *n_steps = steps;
  if (n_gemm) *n_gemm = gemm;
  if (gemm_flops) *gemm_flops = fg;
  if (total_flops) *total_flops = ft;
  return QTN_OK;
}

qtn_status qtn_get_info(const qtn_net* n, qtn_info* out) {
  if (!n || !out) return fail(QTN_EINVAL, "net or out is NULL");
  std::memset(out, 0, sizeof(*out));
  out->n_cones = (int32_t)n->P.cones.size();
  out->p = n->P.p;
  out->dtype = n->c128 ? QTN_C128 : QTN_C64;
  if (!n->P.ordered) return QTN_OK;
  out->max_width = n->P.max_width;
  for (size_t c = 0; c < n->P.cones.size(); ++c) {
    const Cone& C = n->P.cones[c];
    out->n_buckets += (int64_t)C.plain.size();
    out->n_steps += (int64_t)C.buckets.size();
    out->fwd_bytes += C.fwd_bytes_alg;
    out->bwd_bytes += C.bwd_bytes_alg;
    out->fwd_flops += C.fwd_flops;
    for (const Bucket& B : C.plain) {
      double in = 0;
      for (uint32_t m : B.in_mask) in += std::ldexp(1.0, __builtin_popcount(m));
      const double o = std::ldexp(1.0, B.out_rank());
      out->fwd_bytes_bucket += (in + o) * n->elem;
      out->bwd_bytes_bucket += (o + 2 * in) * n->elem;
    }
    out->n_ops_fwd += n->P.cone_fwd_hi[c] + 1 - n->P.cone_fwd_lo[c];
    out->n_ops_grad += (n->P.cone_fwd_hi[c] - n->P.cone_fwd_lo[c]) + (n->P.cone_adj_hi[c] - n->P.cone_adj_lo[c]);
  }
  out->n_items_fwd = (int64_t)(n->P.items_fwd.size() + n->P.small_items_fwd.size() / 2);
  out->n_items_grad = (int64_t)(n->P.items_grad.size() + n->P.small_items_grad.size() / 2);
  out->ws_fwd = ws_layout(n, false).total;
  out->ws_grad = ws_layout(n, true).total;
  for (char l : n->P.cone_lds) out->n_lds_cones += l ? 1 : 0;
  out->lds_window = (int32_t)(n->P.lds_elems * n->elem);
  for (const Cone& C : n->P.cones) {
    for (char r : C.recompute) out->n_recomputed += r ? 1 : 0;
    out->rec_bytes += C.rec_bytes;
    out->arena_keep_all += (size_t)C.keep_all_elems * n->elem;
    out->pinned_bytes += (size_t)((C.dyn_start + 63) / 64 * 64) * n->elem;
    out->max_cone_dynamic = std::max(out->max_cone_dynamic, (size_t)(C.keep_all_elems - C.dyn_start) * n->elem);
  }
  return QTN_OK;
}

qtn_status qtn_cone_stats(const qtn_net* n, int32_t* width, int32_t* n_qubits, int32_t* n_indices, int32_t* n_tensors,
                          int32_t* n_buckets, double* fwd_bytes, double* bwd_bytes) {
  if (!n) return fail(QTN_EINVAL, "net is NULL");
  for (size_t c = 0; c < n->P.cones.size(); ++c) {
    const Cone& C = n->P.cones[c];
    if (width) width[c] = C.width;
    if (n_qubits) n_qubits[c] = C.n_qubits;
    if (n_indices) n_indices[c] = C.n_idx;
    if (n_tensors) n_tensors[c] = (int32_t)C.leaves.size();
    if (n_buckets) n_buckets[c] = (int32_t)C.plain.size();
    if (fwd_bytes) fwd_bytes[c] = C.fwd_bytes_alg;
    if (bwd_bytes) bwd_bytes[c] = C.bwd_bytes_alg;
  }
  return QTN_OK;
}

qtn_status qtn_get_tuning(const qtn_net* n, qtn_tuning* out) {
  if (!n || !out) return fail(QTN_EINVAL, "net or out is NULL");
  out->threads = n->P.tune.threads;
  out->lane_cap = n->P.tune.lane_cap;
  out->seq_max_bits = n->P.tune.seq_max_bits;
  out->tile_blocks = n->P.tune.tile_blocks;
  out->loop_cap = n->P.tune.loop_cap;
  out->grid = n->grid;
  out->lds_kb = n->P.tune.lds_kb;
  out->par_bits = n->P.tune.par_bits;
  out->merge_bits = n->P.tune.merge_bits;
  out->merge_lam_bits = n->P.tune.merge_lam_bits;
  out->lane_low = n->P.tune.lane_low;
  out->fuse_adjoint = n->P.tune.fuse_adjoint;
  out->lds_threads = n->P.tune.lds_threads;
  return QTN_OK;
}

qtn_status qtn_set_tuning(qtn_net* n, const qtn_tuning* t) {
  if (!n || !t) return fail(QTN_EINVAL, "net or tuning is NULL");
  const int th = t->threads;
  if (th != 64 && th != 128 && th != 256 && th != 512) return fail(QTN_EINVAL, "threads must be 64, 128, 256 or 512");
  if (t->lane_cap < 1 || t->lane_cap > 10) return fail(QTN_EINVAL, "lane_cap must be in 1..10");
  if (t->seq_max_bits < 1 || t->seq_max_bits > 31) return fail(QTN_EINVAL, "seq_max_bits must be in 1..31");
  if (t->tile_blocks < 1 || (t->tile_blocks & (t->tile_blocks - 1)))
    return fail(QTN_EINVAL, "tile_blocks must be a power of two");
  if (t->loop_cap < 0 || t->loop_cap > 31) return fail(QTN_EINVAL, "loop_cap must be in 0..31");
  if (t->grid < 0) return fail(QTN_EINVAL, "grid must be >= 0");
  if (t->lds_kb < 0 || t->lds_kb > 128) return fail(QTN_EINVAL, "lds_kb must be in 0..128");
  if (t->par_bits < 8 || t->par_bits > 24) return fail(QTN_EINVAL, "par_bits must be in 8..24");
  if (t->merge_bits < 0 || t->merge_bits > 16) return fail(QTN_EINVAL, "merge_bits must be in 0..16");
  if (t->merge_lam_bits < 0 || t->merge_lam_bits > 16) return fail(QTN_EINVAL, "merge_lam_bits must be in 0..16");
  if (t->lane_low != 0 && t->lane_low != 1) return fail(QTN_EINVAL, "lane_low must be 0 or 1");
  if (t->fuse_adjoint < 0 || t->fuse_adjoint > 3) return fail(QTN_EINVAL, "fuse_adjoint must be 0, 1, 2 or 3");
  if (t->lds_threads != 64 && t->lds_threads != 128 && t->lds_threads != 256 && t->lds_threads != 512)
    return fail(QTN_EINVAL, "lds_threads must be 64, 128, 256 or 512");
  n->P.tune.threads = th;
  n->P.tune.lane_low = t->lane_low;
  n->P.tune.fuse_adjoint = t->fuse_adjoint;
  n->P.tune.lds_threads = t->lds_threads;
  n->P.tune.par_bits = t->par_bits;
  n->P.tune.merge_bits = t->merge_bits;
  n->P.tune.merge_lam_bits = t->merge_lam_bits;
  n->P.tune.lane_cap = t->lane_cap;
  n->P.tune.seq_max_bits = t->seq_max_bits;
  n->P.tune.tile_blocks = t->tile_blocks;
  n->P.tune.loop_cap = t->loop_cap;
  n->P.tune.lds_kb = t->lds_kb;
  n->grid = t->grid ? t->grid : 8 * n->ctx->n_cu;
  if (!n->P.ordered) return QTN_OK;
  return rebuild_programs(n);
}

qtn_status qtn_autotune(qtn_net* n, int32_t with_grad, void* ws, size_t ws_bytes, void* stream, int32_t reps,
                        qtn_tuning* best_out) {
  qtn_status s = check_ready(n, ws, ws_bytes, with_grad != 0);
  if (s != QTN_OK) return s;
  if (reps < 1) reps = 3;
  hipStream_t st = (hipStream_t)stream;
  qtn_tuning base;
  qtn_get_tuning(n, &base);
  hipEvent_t e0, e1;
  HIPCHECK(hipEventCreate(&e0));
  HIPCHECK(hipEventCreate(&e1));
  // time one candidate: a warm sweep (re-captures the graph) then `reps`
  auto timed = [&](const qtn_tuning& t, double* ms_out) -> qtn_status {
    qtn_status r;
    if ((r = qtn_set_tuning(n, &t)) != QTN_OK) return r;
    if (ws_layout(n, with_grad != 0).total > ws_bytes) {  // needs a larger workspace: not a candidate here
      *ms_out = 1e300;
      return QTN_OK;
    }
    if ((r = check_ready(n, ws, ws_bytes, with_grad != 0)) != QTN_OK) return r;
    if ((r = run_sweep(n, QTN_BATCHED, with_grad != 0, ws, ws_bytes, st, nullptr, true)) != QTN_OK) return r;
    // one timed sweep sizes the replay count: about 25 ms of sweeps per
    // candidate (short sweeps are noisy), at least `reps`, at most 200
    float ms = 0;
    int k_reps = 1;
    for (int pass = 0; pass < 2; ++pass) {
      HIPCHECK(hipEventRecord(e0, st));
      for (int k = 0; k < k_reps; ++k)
        if ((r = run_sweep(n, QTN_BATCHED, with_grad != 0, ws, ws_bytes, st, nullptr, false)) != QTN_OK) return r;
      HIPCHECK(hipEventRecord(e1, st));
      HIPCHECK(hipEventSynchronize(e1));
      if (sweep_flag(n)) return fail(QTN_EDEVICE, "persistent sweep gave up waiting on a dependency");
      HIPCHECK(hipEventElapsedTime(&ms, e0, e1));
      ms /= (float)k_reps;
      if (pass == 0) k_reps = std::max(reps, std::min(200, (int)std::ceil(25.0 / std::max(ms, 1e-3f))));
    }
    *ms_out = ms;
    return QTN_OK;
  };
  // coordinate descent over four groups of parameters: workgroup shape,
  // split thresholds of wide buckets, merging of small buckets, the kernel of
  // the LDS-resident cones
  double best_ms = 1e300;
  qtn_tuning best = base;
  for (int stage = 0; stage < 4 && s == QTN_OK; ++stage) {
    std::vector<qtn_tuning> cand;
    const qtn_tuning b0 = best;
    if (stage == 0) {
      for (int th : {64, 128, 256, 512})
        for (int lc : {6, 7, 8}) {
          if ((1 << lc) > th) continue;
          qtn_tuning t = b0;
          t.threads = th;
          t.lane_cap = lc;
          t.grid = 0;
          cand.push_back(t);
        }
    } else if (stage == 1) {
      for (int sq : {12, 14, 16})
        for (int tb : {16, 64, 128}) {
          qtn_tuning t = b0;
          t.seq_max_bits = sq;
          t.tile_blocks = tb;
          cand.push_back(t);
        }
    } else if (stage == 3) {
      // LDS-resident cones: workgroup size and LDS window cap
      for (int lt : {128, 256, 512})
        for (int kb : {64, 96}) {
          qtn_tuning t = b0;
          t.lds_threads = lt;
          t.lds_kb = kb;
          cand.push_back(t);
        }
    } else {
      for (auto mm : {std::pair<int, int>{0, 0}, {8, 6}, {10, 7}, {12, 7}, {12, 8}}) {
        qtn_tuning t = b0;
        t.merge_bits = mm.first;
        t.merge_lam_bits = mm.second;
        cand.push_back(t);
      }
    }
    for (const qtn_tuning& t : cand) {
      double ms = 0;
      if ((s = timed(t, &ms)) != QTN_OK) break;
      if (ms < best_ms) {
        best_ms = ms;
        best = t;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (s != QTN_OK) return s;
  s = qtn_set_tuning(n, &best);
  n->kernel_ms_sum = 0;
  n->kernel_count = 0;
  if (best_out) *best_out = best;
  return s;
}

qtn_status qtn_time_wide_ops(qtn_net* n, int32_t with_grad, int32_t min_width, void* ws, size_t ws_bytes,
                             void* stream, int32_t reps, double* bytes_out, double* ms_out, int64_t* n_ops_out) {
  qtn_status s = check_ready(n, ws, ws_bytes, with_grad != 0);
  if (s != QTN_OK) return s;
  if (reps < 1) reps = 1;
  hipStream_t st = (hipStream_t)stream;
  HIPCHECK(hipSetDevice(n->ctx->device));
  const WsLayout L = ws_layout(n, with_grad != 0);
  Env env = make_env(n, static_cast<char*>(ws), L);
  hipEvent_t e0, e1;
  HIPCHECK(hipEventCreate(&e0));
  HIPCHECK(hipEventCreate(&e1));
  double bytes = 0, ms_tot = 0;
  int64_t cnt = 0;
  (void)hipGetLastError();
  for (size_t c = 0; c < n->P.cones.size() && s == QTN_OK; ++c) {
    std::vector<std::pair<int32_t, int32_t>> ranges = {{n->P.cone_fwd_lo[c], n->P.cone_fwd_hi[c]}};
    if (with_grad) ranges.push_back({n->P.cone_adj_lo[c], n->P.cone_adj_hi[c]});
    for (auto& r : ranges)
      for (int32_t o = r.first; o < r.second; ++o) {
        const OpDesc& d = n->P.ops[o];
        if ((d.kind != OP_CONTRACT && d.kind != OP_ADJOINT) || d.nbits - 1 < min_width) continue;
        double b = d.kind == OP_CONTRACT ? std::ldexp(1.0, __builtin_popcount(d.out_mask)) : 0.0;
        for (int i = 0; i < d.n_in; ++i)
          b += std::ldexp(1.0, __builtin_popcount(d.in_mask[i])) * (((d.adj_sel >> i) & 1u) ? 2 : 1);
        b *= n->elem;
        HIPCHECK(launch_op(n->c128, n->d_ops, d, o, env, n->P.tune.threads, 4096, st));  // warm
        HIPCHECK(hipEventRecord(e0, st));
        for (int k = 0; k < reps; ++k) HIPCHECK(launch_op(n->c128, n->d_ops, d, o, env, n->P.tune.threads, 4096, st));
        HIPCHECK(hipEventRecord(e1, st));
        HIPCHECK(hipEventSynchronize(e1));
        float ms = 0;
        HIPCHECK(hipEventElapsedTime(&ms, e0, e1));
        bytes += b;
        ms_tot += ms / reps;
        ++cnt;
      }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (bytes_out) *bytes_out = bytes;
  if (ms_out) *ms_out = ms_tot;
  if (n_ops_out) *n_ops_out = cnt;
  return QTN_OK;
}

qtn_status qtn_time_wide_sweep(qtn_net* n, int32_t with_grad, int32_t min_width, int32_t max_width, int32_t kinds,
                               void* ws, size_t ws_bytes, void* stream, int32_t reps, double* bytes_out,
                               double* op_bytes_out, double* ms_out, int64_t* n_ops_out, int64_t* n_items_out) {
  qtn_status s = check_ready(n, ws, ws_bytes, with_grad != 0);
  if (s != QTN_OK) return s;
  if (reps < 1) return fail(QTN_EINVAL, "reps must be >= 1");
  const bool grad = with_grad != 0;
  // the ops of buckets with output rank >= min_width, in each cone's program
  // order, as a queue of their own
  std::vector<char> in_prog(n->P.ops.size(), 0);  // 1: forward op, 2: adjoint-sweep op
  for (size_t c = 0; c < n->P.cones.size(); ++c) {
    for (int32_t o = n->P.cone_fwd_lo[c]; o < n->P.cone_fwd_hi[c]; ++o) in_prog[o] = 1;
    if (grad)
      for (int32_t o = n->P.cone_adj_lo[c]; o < n->P.cone_adj_hi[c]; ++o) in_prog[o] = 2;
  }
  double bytes = 0;
  int64_t cnt = 0;
  if (max_width <= 0) max_width = MAXBITS;
  if (kinds == 0) kinds = 7;
  auto keep = [&](int32_t o) {
    const OpDesc& d = n->P.ops[o];
    if (!in_prog[o] || (d.kind != OP_CONTRACT && d.kind != OP_ADJOINT)) return false;
    if (d.nbits - 1 < min_width || d.nbits - 1 > max_width) return false;
    // forward contraction, one-input adjoint pass (or a recomputation in the
    // adjoint sweep), fused adjoint
    const int kind = d.kind == OP_ADJOINT ? 4 : (in_prog[o] == 1 ? 1 : 2);
    return (kinds & kind) != 0;
  };
  for (size_t o = 0; o < n->P.ops.size(); ++o) {
    if (!keep((int32_t)o)) continue;
    const OpDesc& d = n->P.ops[o];
    double b = d.kind == OP_CONTRACT ? std::ldexp(1.0, __builtin_popcount(d.out_mask)) : 0.0;
    for (int i = 0; i < d.n_in; ++i)
      b += std::ldexp(1.0, __builtin_popcount(d.in_mask[i])) * (((d.adj_sel >> i) & 1u) ? 2 : 1);
    bytes += b * n->elem;
    ++cnt;
  }
  // algorithmic bytes of the selected contraction steps, as the sweep's
  // totals count them: forward, every input read and the output written;
  // adjoint, the output adjoint and every stored input read and every input
  // adjoint written (queued cones only: LDS-resident ones are not in a
  // sub-sweep)
  double alg = 0;
  for (size_t c = 0; c < n->P.cones.size(); ++c) {
    if (!n->P.cone_lds.empty() && n->P.cone_lds[c]) continue;
    for (const Bucket& B : n->P.cones[c].buckets) {
      const int w = B.nbits() - 1;
      if (w < min_width || w > max_width) continue;
      double in = 0;
      for (uint32_t m : B.in_mask) in += std::ldexp(1.0, __builtin_popcount(m));
      const double out = std::ldexp(1.0, B.out_rank());
      if (kinds & 1) alg += in + out;
      if (grad && (kinds & 6)) alg += out + 2 * in;
    }
  }
  alg *= n->elem;
  Queue q;
  try {
    build_queue(n->P, grad, keep, q);
  } catch (const std::bad_alloc&) {
    return fail(QTN_ENOMEM, "host allocation failed");
  }
  if (bytes_out) *bytes_out = alg;
  if (op_bytes_out) *op_bytes_out = bytes;
  if (n_ops_out) *n_ops_out = cnt;
  if (n_items_out) *n_items_out = (int64_t)q.items.size();
  if (ms_out) *ms_out = 0;
  if (q.items.empty()) return QTN_OK;
  if (q.init.size() > (size_t)std::max(n->prog[0].n_nodes, n->prog[1].n_nodes))
    return fail(QTN_EUNSUPPORTED, "sub-sweep has more queue nodes than the workspace holds");
  hipStream_t st = (hipStream_t)stream;
  HIPCHECK(hipSetDevice(n->ctx->device));
  DevProg pg;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto release = [&]() {
    (void)hipFree(pg.items);
    (void)hipFree(pg.succ);
    (void)hipFree(pg.init);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  };
  hipError_t e = upload(&pg.items, q.items);
  if (e == hipSuccess) e = upload(&pg.succ, q.succ);
  if (e == hipSuccess) e = upload(&pg.init, q.init);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e != hipSuccess) {
    release();
    return fail(QTN_EDEVICE, std::string("sub-sweep setup: ") + hipGetErrorString(e));
  }
  const WsLayout L = ws_layout(n, grad);
  char* w = static_cast<char*>(ws);
  Env env = make_env(n, w, L);
  int32_t* ctl = reinterpret_cast<int32_t*>(w + L.ctl_off);
  const int n_items = (int)q.items.size();
  const int grid = std::max(1, std::min<int>(n->grid, n_items));
  const size_t lds_bytes = (size_t)n->P.lds_elems * n->elem;
  double tot = 0;
  int32_t flag = 0;
  (void)hipGetLastError();
  for (int r = 0; r <= reps && e == hipSuccess; ++r) {  // the first run warms up
    e = launch_reset(ctl, pg.init, (int)q.init.size(), st);
    if (e == hipSuccess) e = hipEventRecord(e0, st);
    if (e == hipSuccess)
      e = launch_persistent(n->c128, n->has_wide, n->max_nin, n->d_ops, pg.items, n_items, pg.succ, ctl, env,
                            n->P.tune.threads, grid, lds_bytes, kSpinLimit, st);
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e == hipSuccess) e = hipMemcpy(&flag, ctl + 1, sizeof(flag), hipMemcpyDeviceToHost);
    if (e == hipSuccess && flag) break;
    if (r > 0) tot += ms;
  }
  release();
  if (e != hipSuccess) return fail(QTN_EDEVICE, std::string("sub-sweep: ") + hipGetErrorString(e));
  if (flag) return fail(QTN_EDEVICE, "sub-sweep gave up waiting on a dependency");
  if (ms_out) *ms_out = tot / reps;
  return QTN_OK;
}

qtn_status qtn_time_persistent(qtn_net* n, int32_t with_grad, void* ws, size_t ws_bytes, void* stream,
                               int32_t reps, double* ms_out) {
  qtn_status s = check_ready(n, ws, ws_bytes, with_grad != 0);
  if (s != QTN_OK) return s;
  if (reps < 1) return fail(QTN_EINVAL, "reps must be >= 1");
  hipStream_t st = (hipStream_t)stream;
  HIPCHECK(hipSetDevice(n->ctx->device));
  hipEvent_t e0, e1;
  HIPCHECK(hipEventCreate(&e0));
  HIPCHECK(hipEventCreate(&e1));
  double tot = 0;
  for (int r = 0; r <= reps && s == QTN_OK; ++r) {  // the first sweep warms up
    s = enqueue_sweep(n, QTN_BATCHED, with_grad != 0, ws, st, nullptr, e0, e1);
    if (s != QTN_OK) break;
    hipError_t e = hipEventSynchronize(e1);
    float ms = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) s = fail(QTN_EDEVICE, std::string("persistent kernel timing: ") + hipGetErrorString(e));
    if (r > 0) tot += ms;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (s != QTN_OK) return s;
  HIPCHECK(hipStreamSynchronize(st));
  if (sweep_flag(n)) return fail(QTN_EDEVICE, "persistent sweep gave up waiting on a dependency");
  if (ms_out) *ms_out = tot / reps;
  return QTN_OK;
}

qtn_status qtn_cost_model(int32_t n_vertices, int32_t n_edges, const int32_t* edges, int32_t p,
                          qtn_net_variant variant, qtn_order_kind kind, int32_t n_repeats, double temperature,
                          uint64_t seed, qtn_cost* out) {
  return qtn_cost_model_order(n_vertices, n_edges, edges, p, variant, kind, n_repeats, temperature, seed, out,
                              nullptr, 0);
}

qtn_status qtn_cost_model_order(int32_t n_vertices, int32_t n_edges, const int32_t* edges, int32_t p,
                                qtn_net_variant variant, qtn_order_kind kind, int32_t n_repeats, double temperature,
                                uint64_t seed, qtn_cost* out, int32_t* order_out, int32_t order_cap) {
  if (!out) return fail(QTN_EINVAL, "out is NULL");
  if (order_out && order_cap < 0) return fail(QTN_EINVAL, "order_cap must be >= 0");
  if (variant < QTN_NET_DEFAULT || variant > QTN_NET_DIAGONAL_ZZ) return fail(QTN_EINVAL, "unknown network variant");
  if (kind != QTN_ORDER_MIN_DEGREE && kind != QTN_ORDER_MIN_FILL) return fail(QTN_EINVAL, "unknown order kind");
  if (n_repeats < 0 || !(temperature >= 0.0) || !std::isfinite(temperature))
    return fail(QTN_EINVAL, "n_repeats must be >= 0 and temperature finite and >= 0");
  std::string err = validate_graph(n_vertices, n_edges, edges, p);
  if (!err.empty()) return fail(QTN_EINVAL, err);
  try {
    std::vector<std::pair<int32_t, int32_t>> E;
    for (int e = 0; e < n_edges; ++e) E.push_back({edges[2 * e], edges[2 * e + 1]});
    OrderOptions O;
    O.kind = (int)kind;
    O.repeats = n_repeats;
    O.temperature = temperature;
    O.seed = seed;
    const auto t0 = std::chrono::steady_clock::now();
    std::vector<int> order;
    const CostEstimate c = cost_model(n_vertices, E, p, (int)variant, O, order_out ? &order : nullptr);
    out->order_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    out->n_indices = c.n_indices;
    out->n_tensors = c.n_tensors;
    out->width = c.width;
    out->log2_ops = c.log2_ops;
    if (order_out) {
      if (order_cap < c.n_indices)
        return fail(QTN_EINVAL, "order_out holds " + std::to_string(order_cap) + " entries, the network has " +
                                    std::to_string(c.n_indices) + " indices");
      std::copy(order.begin(), order.end(), order_out);
    }
    return QTN_OK;
  } catch (const std::bad_alloc&) {
    return fail(QTN_ENOMEM, "host allocation failed");
  }
}

qtn_status qtn_copy_bandwidth(qtn_ctx* ctx, void* buf, size_t bytes, void* stream, int32_t reps, double* gbps_out) {
  if (!ctx) return fail(QTN_EINVAL, "context is NULL");
  if (ctx->device < 0) return fail(QTN_ESTATE, "host-only context has no device");
  if (!buf || bytes < 32 || reps < 1) return fail(QTN_EINVAL, "need a device buffer of >= 32 bytes and reps >= 1");
  if (reinterpret_cast<uintptr_t>(buf) % 16) return fail(QTN_EINVAL, "buffer must be 16-byte aligned");
  HIPCHECK(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  const size_t n16 = bytes / 32;  // 16-byte words per half
  char* src = static_cast<char*>(buf);
  char* dst = src + n16 * 16;
  hipEvent_t e0, e1;
  HIPCHECK(hipEventCreate(&e0));
  HIPCHECK(hipEventCreate(&e1));
  // the best of a few launch shapes: 1, 2 or 4 loads in flight per thread,
  // 4 to 32 256-thread workgroups per compute unit
  double best = 0;
  hipError_t e = hipSuccess;
  for (int unroll : {1, 2, 4})
    for (int per_cu : {4, 8, 16, 32}) {
      const int grid = per_cu * ctx->n_cu;
      e = launch_copy(src, dst, n16, grid, unroll, st);
      if (e == hipSuccess) e = hipEventRecord(e0, st);
      for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch_copy(src, dst, n16, grid, unroll, st);
      if (e == hipSuccess) e = hipEventRecord(e1, st);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e != hipSuccess) break;
      best = std::max(best, 2.0 * (double)(n16 * 16) * reps / (ms * 1e-3) / 1e9);
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return fail(QTN_EDEVICE, std::string("copy kernel: ") + hipGetErrorString(e));
  if (gbps_out) *gbps_out = best;
  return QTN_OK;
}

qtn_status qtn_get_band_tuning(const qtn_net* n, qtn_band_tuning* out) {
  if (!n || !out) return fail(QTN_EINVAL, "net or out is NULL");
  for (int b = 0; b < QTN_BANDS; ++b) {
    out[b].par_bits = n->P.tune.band[b].par_bits;
    out[b].tile_blocks = n->P.tune.band[b].tile_blocks;
    out[b].loop_cap = n->P.tune.band[b].loop_cap;
  }
  return QTN_OK;
}

qtn_status qtn_set_band_tuning(qtn_net* n, const qtn_band_tuning* in) {
  if (!n || !in) return fail(QTN_EINVAL, "net or in is NULL");
  for (int b = 0; b < QTN_BANDS; ++b) {
    const qtn_band_tuning& t = in[b];
    if (t.par_bits != 0 && (t.par_bits < 8 || t.par_bits > 24)) return fail(QTN_EINVAL, "band par_bits must be 0 or 8..24");
    if (t.tile_blocks < 0 || (t.tile_blocks & (t.tile_blocks - 1)))
      return fail(QTN_EINVAL, "band tile_blocks must be 0 or a power of two");
    if (t.loop_cap < 0 || t.loop_cap > 31) return fail(QTN_EINVAL, "band loop_cap must be in 0..31");
  }
  TuneParams::Band old[TuneParams::kBands];
  for (int b = 0; b < QTN_BANDS; ++b) {
    old[b] = n->P.tune.band[b];
    n->P.tune.band[b].par_bits = in[b].par_bits;
    n->P.tune.band[b].tile_blocks = in[b].tile_blocks;
    n->P.tune.band[b].loop_cap = in[b].loop_cap;
  }
  if (!n->P.ordered) return QTN_OK;
  qtn_status s = rebuild_programs(n);
  if (s != QTN_OK) {
    const std::string msg = qtn_last_error();
    for (int b = 0; b < QTN_BANDS; ++b) n->P.tune.band[b] = old[b];
    (void)rebuild_programs(n);
    return fail(s, msg);
  }
  return QTN_OK;
}

qtn_status qtn_autotune_bands(qtn_net* n, int32_t with_grad, void* ws, size_t ws_bytes, void* stream, int32_t reps,
                              qtn_band_tuning* best_out, double* ms_out) {
  qtn_status s = check_ready(n, ws, ws_bytes, with_grad != 0);
  if (s != QTN_OK) return s;
  if (reps < 1) reps = 2;
  // widths (output ranks) of each band's buckets: union bits - 1
  const int lo_w[QTN_BANDS] = {n->P.tune.seq_max_bits, 20, 24};
  const int hi_w[QTN_BANDS] = {19, 23, MAXBITS};
  qtn_band_tuning cur[QTN_BANDS];
  qtn_get_band_tuning(n, cur);
  for (int b = 0; b < QTN_BANDS && s == QTN_OK; ++b) {
    if (lo_w[b] > hi_w[b]) continue;
    bool any = false;
    for (const OpDesc& d : n->P.ops)
      any |= (d.kind == OP_CONTRACT || d.kind == OP_ADJOINT) && d.nbits - 1 >= lo_w[b] && d.nbits - 1 <= hi_w[b];
    if (!any) continue;
    double best = 1e300;
    qtn_band_tuning keep = cur[b];
    for (int pb : {19, 21, 23})
      for (int tb : {64, 128, 256}) {
        cur[b].par_bits = pb;
        cur[b].tile_blocks = tb;
        cur[b].loop_cap = 0;
        if (qtn_set_band_tuning(n, cur) != QTN_OK) continue;  // no valid plan with these tiles
        if (ws_layout(n, with_grad != 0).total > ws_bytes) continue;
        if ((s = check_ready(n, ws, ws_bytes, with_grad != 0)) != QTN_OK) break;
        double bytes = 0, ms = 0;
        s = qtn_time_wide_sweep(n, with_grad, lo_w[b], hi_w[b], 7, ws, ws_bytes, stream, reps, &bytes, nullptr, &ms,
                                nullptr, nullptr);
        if (s != QTN_OK) break;
        if (ms < best) {
          best = ms;
          keep = cur[b];
        }
      }
    cur[b] = keep;
  }
  if (s == QTN_OK) s = qtn_set_band_tuning(n, cur);
  if (s != QTN_OK) return s;
  n->kernel_ms_sum = 0;
  n->kernel_count = 0;
  if (best_out) qtn_get_band_tuning(n, best_out);
  if (ms_out) return qtn_time_persistent(n, with_grad, ws, ws_bytes, stream, reps, ms_out);
  return QTN_OK;
}

qtn_status qtn_set_sweep_timing(qtn_net* n, int32_t on) {
  if (!n) return fail(QTN_EINVAL, "net is NULL");
  n->sweep_timing = on != 0;
  return QTN_OK;
}

qtn_status qtn_kernel_time(qtn_net* n, double* ms_sum, int64_t* count, int32_t reset) {
  if (!n) return fail(QTN_EINVAL, "net is NULL");
  if (ms_sum) *ms_sum = n->kernel_ms_sum;
  if (count) *count = n->kernel_count;
  if (reset) {
    n->kernel_ms_sum = 0;
    n->kernel_count = 0;
  }
  return QTN_OK;
}

qtn_status qtn_set_memory_budget(qtn_net* n, size_t bytes) {
  if (!n) return fail(QTN_EINVAL, "net is NULL");
  n->P.mem_budget = (int64_t)(bytes / (size_t)n->elem);
  if (!n->P.ordered) return QTN_OK;
  qtn_status s = rebuild_programs(n);
  if (s == QTN_EUNSUPPORTED) {  // the builder reports an unreachable budget this way
    n->P.mem_budget = 0;
    (void)rebuild_programs(n);
    return fail(QTN_ENOMEM, "memory budget of " + std::to_string(bytes) + " bytes cannot be met");
  }
  return s;
}

qtn_status qtn_validate_plan(const qtn_net* n) {
  if (!n) return fail(QTN_EINVAL, "net is NULL");
  if (!n->P.ordered) return fail(QTN_ESTATE, "qtn_order has not been called");
  std::string err = validate_plan(n->P);
  return err.empty() ? QTN_OK : fail(QTN_EINVAL, err);
}

void qtn_net_free(qtn_net* n) {
  if (!n) return;
  if (n->ctx->device < 0) {
    std::free(n->h_leafvals);
    delete n;
    return;
  }
  (void)hipSetDevice(n->ctx->device);
  if (n->ev_done) (void)hipEventSynchronize(n->ev_done);
  free_device_plan(n);
  (void)hipFree(n->d_leafvals);
  if (n->h_leafvals) (void)hipHostFree(n->h_leafvals);
  if (n->h_fin) (void)hipHostFree(n->h_fin);
  if (n->ev_k0) (void)hipEventDestroy(n->ev_k0);
  if (n->ev_k1) (void)hipEventDestroy(n->ev_k1);
  if (n->ev_done) (void)hipEventDestroy(n->ev_done);
  delete n;
}

}  // extern "C"
