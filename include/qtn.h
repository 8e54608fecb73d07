/* qtn.h -- C ABI of the MI355X (gfx950) QAOA-MaxCut light-cone tensor-network
 * library.
 *
 * What it computes (Lykov & Alexeev, "Importance of Diagonal Gates in Tensor
 * Network Simulations"):
 *   * the MaxCut cost C = 1/2 sum_{(j,k) in E} (1 - Z_j Z_k) and the QAOA state
 *     |gamma beta> = prod_l U_B(beta_l) U_C(gamma_l) |+>^N with
 *     U_C(gamma) = exp(-i gamma C), U_B(beta) = exp(-i beta sum_q X_q)
 *     (Section II, eq. qaoa1; layer 1 first, cost before mixer);
 *   * E = <gamma beta| C |gamma beta> = sum over edges of (1 - <Z_j Z_k>)/2, each
 *     edge term from its own light-cone tensor network (Section II);
 *   * each network is built with the ZZ phase gates as rank-2 diagonal tensors
 *     that add no index (Section IV.B, eq. example) and contracted by bucket
 *     elimination (Section III.B, eq. tn);
 *   * dE/dgamma_l and dE/dbeta_l by a reverse sweep over the same buckets.
 *
 * Conventions: all entry points return a qtn_status; on anything but QTN_OK
 * qtn_last_error() returns a message (thread-local, valid until the next call
 * on the same thread).  No C++ exception crosses this interface.  Host
 * pointers are only read during the call (inputs are copied).  Device
 * pointers (workspace, zz_out) are owned by the caller and must stay valid
 * until the work queued on `stream` has finished.  `stream` is a hipStream_t
 * (NULL = the legacy default stream).  Every call is asynchronous on `stream`
 * except when it writes host outputs, in which case it synchronises `stream`
 * before returning.  A qtn_net must not be used by two threads at once.
 */
#ifndef QTN_H
#define QTN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qtn_ctx qtn_ctx;
typedef struct qtn_net qtn_net;

typedef enum {
  QTN_OK = 0,
  QTN_EINVAL = 1,       /* bad argument: graph, depth, angle, pointer, mode */
  QTN_ENOMEM = 2,       /* workspace smaller than qtn_workspace_size(), or host/device allocation failed */
  QTN_EDEVICE = 3,      /* a HIP call failed, or a kernel reported an error */
  QTN_EUNSUPPORTED = 4, /* plan exceeds a kernel limit (width > 30, > 8 inputs per bucket) */
  QTN_ESTATE = 5        /* call out of order (e.g. contract before qtn_order / qtn_set_params) */
} qtn_status;

typedef enum { QTN_C64 = 0, QTN_C128 = 1 } qtn_dtype;          /* complex64 (FP32 accumulate) or complex128 */
typedef enum { QTN_ORDER_MIN_DEGREE = 0, QTN_ORDER_MIN_FILL = 1 } qtn_order_kind;
typedef enum { QTN_PLAIN = 0, QTN_BATCHED = 1 } qtn_mode;
/* QTN_PLAIN: host loop over edges, one kernel launch per bucket step.
 * QTN_BATCHED: every light cone in one persistent launch fed by a device work
 * queue, captured once as a hipGraph and replayed. */

/* Kernel tile parameters (see qtn_set_tuning / qtn_autotune). */
typedef struct {
  int32_t threads;      /* workgroup size: 64, 128, 256 or 512 */
  int32_t lane_cap;     /* max union bits mapped to the lanes of one sub-block (1..10) */
  int32_t seq_max_bits; /* buckets with more union bits than this are split across workgroups */
  int32_t tile_blocks;  /* blocks of a split bucket handled by one queue item (power of two) */
  int32_t loop_cap;     /* summed bits looped inside a thread before partial sums go to atomics */
  int32_t grid;         /* persistent workgroups (0: 8 per compute unit; 1: one workgroup takes the queue's
                           items in order, a deterministic schedule in which no item waits) */
  int32_t lds_kb;       /* LDS window (KiB, <= 128) for light cones that run LDS-resident in the batched sweep: leaf
                           tables, intermediates and adjoints of such a cone never leave LDS (0: none) */
  int32_t par_bits;     /* a split bucket aims at >= 2^par_bits threads before summing in per-thread loops (8..24) */
  int32_t merge_bits;   /* a bucket is merged into its consumer while the merged step's union has <= merge_bits
                           bits (0: one step per bucket; at most 16) */
  int32_t merge_lam_bits; /* ... and its leaf-product table carries <= merge_lam_bits indices (0..16) */
  int32_t lane_low;     /* 1: split buckets map lanes to their lowest union bits, summed or not (contiguous input
                           reads, partial sums combined across lanes); 0: to their lowest output bits first */
  int32_t fuse_adjoint; /* 1: the adjoint of a split bucket computes every input adjoint in one pass over its
                           union (output adjoint and inputs read once) where the loop bits can be chosen so
                           that no output needs atomics per step; 2: also the other buckets, summed tile by tile
                           in LDS (slower on MI355X: LDS atomics); 3: the other buckets of complex64 nets with
                           inputs that each lack part of the union (outer products) in one pass with register
                           slots, one output sum per loop step (slower on MI355X where many partial sums remain
                           for atomics); 0: one pass per input adjoint */
  int32_t lds_threads;  /* workgroup size (64, 128, 256 or 512) of the kernel that runs the light cones whose whole
                           program fits the LDS window (lds_kb), one workgroup per cone */
} qtn_tuning;

typedef struct {
  int32_t n_cones;          /* = number of edges */
  int32_t p;
  int32_t max_width;        /* largest bucket output rank over all cones */
  int32_t dtype;            /* qtn_dtype */
  int64_t n_buckets;        /* total buckets over all cones (one per index) */
  int64_t n_ops_fwd;        /* device ops of the forward program */
  int64_t n_ops_grad;       /* device ops of the forward + adjoint program */
  int64_t n_items_fwd, n_items_grad;  /* work items of the batched sweep: persistent-queue items plus one per
                                         LDS-resident light cone */
  double fwd_bytes;         /* algorithmic bytes of one forward sweep (each input read once, output written once) */
  double bwd_bytes;         /* algorithmic bytes of the adjoint sweep */
  double fwd_flops;         /* complex multiply = 6, add = 2 */
  size_t ws_fwd, ws_grad;   /* workspace bytes: forward only / forward + gradient */
  int32_t n_lds_cones;      /* light cones that run LDS-resident in the batched sweep */
  int32_t lds_window;       /* bytes of LDS window each persistent workgroup reserves for them */
  int64_t n_recomputed;     /* bucket outputs dropped after the forward sweep and recomputed in the adjoint */
  double rec_bytes;         /* extra bytes of those recomputations per gradient sweep (not algorithmic) */
  size_t arena_keep_all;    /* arena bytes the gradient sweep would need keeping every output */
  int64_t n_steps;          /* contraction steps over all cones (buckets after merging small ones) */
  double fwd_bytes_bucket;  /* the same counts per bucket of the elimination order (one bucket per index, before
                               merging): forward s * sum_b (sum_t 2^rank(t) + 2^rank(out_b)) over intermediate
                               inputs t (rank <= 2 leaves left out); adjoint s * sum_b (2^rank(out_b) + 2 sum_t
                               2^rank(t)) (read the output adjoint and the stored inputs, write the input adjoints) */
  double bwd_bytes_bucket;
  size_t pinned_bytes;      /* arena bytes of every cone's leaf tables and their adjoints (never shared) */
  size_t max_cone_dynamic;  /* largest arena bytes one cone needs beyond them, keeping every output; a memory
                               budget below pinned_bytes + this makes the planner recompute */
} qtn_info;

/* Context bound to HIP device `device` (hipSetDevice is called on it).  Owns a
 * private stream used only for graph capture.  device = QTN_HOST_ONLY gives a
 * planning-only context: build, order, sizes, statistics and plan validation
 * work without a GPU; contractions return QTN_ESTATE. */
#define QTN_HOST_ONLY (-1)
qtn_status qtn_create(int device, qtn_ctx** out);
void qtn_destroy(qtn_ctx* ctx);
const char* qtn_last_error(void);

/* Network for MaxCut on the graph with vertices 0..n_vertices-1 and edge list
 * edges[2*e], edges[2*e+1] (int32, host).  QAOA depth p >= 1.  One light cone
 * per edge (Section II).  Rejects ids out of range, self-loops, duplicate edges
 * (QTN_EINVAL).  No device memory is allocated. */
qtn_status qtn_build(qtn_ctx* ctx, int32_t n_vertices, int32_t n_edges, const int32_t* edges, int32_t p,
                     qtn_dtype dtype, qtn_net** out);

/* Greedy elimination order of every light cone (Section III.B: the order fixes
 * the largest intermediate).  Host work, independent of gamma and beta.
 * Builds the bucket plan and uploads it (the only device allocation of the
 * library).  *max_width_out (nullable) receives the contraction width. */
qtn_status qtn_order(qtn_net* net, qtn_order_kind kind, int32_t* max_width_out);

/* Randomized greedy order (the paper's order finder, Section V, is a
 * randomized greedy run n_repeats times at a temperature): besides the
 * deterministic greedy run, n_repeats runs pick the next index among all
 * candidates with probability proportional to exp(-(score - min score) /
 * temperature) (score: degree or fill-in), seeded by `seed` and the cone
 * index; the run with the least work (sum over buckets of 2^|union|) is kept
 * per cone.  n_repeats = 0 is qtn_order.  Same effects as qtn_order. */
qtn_status qtn_order_rgreedy(qtn_net* net, qtn_order_kind kind, int32_t n_repeats, double temperature,
                             uint64_t seed, int32_t* max_width_out);

/* Bytes of device workspace that qtn_contract (with_grad = 0) or
 * qtn_energy_grad (with_grad = 1) need.  Buffers share memory by lifetime, so
 * both sweeps use the same arena. */
qtn_status qtn_workspace_size(const qtn_net* net, int32_t with_grad, size_t* bytes_out);

/* gamma[p], beta[p] (host, float64, finite).  Leaf tensor values are computed
 * on the host in float64 and cast to the network dtype. */
qtn_status qtn_set_params(qtn_net* net, const double* gamma, const double* beta);

/* Contract every light cone.  workspace: device, >= qtn_workspace_size(.,0)
 * bytes, 256-byte aligned.  zz_out (device, nullable): n_edges complex values
 * <Z_j Z_k> in the network dtype (interleaved re, im).  energy_out (host,
 * nullable): E in float64; when given the call synchronises `stream`. */
qtn_status qtn_contract(qtn_net* net, qtn_mode mode, void* workspace, size_t ws_bytes, void* stream, void* zz_out,
                        double* energy_out);

/* Forward sweep plus the adjoint sweep.  energy_out, dgamma_out[p], dbeta_out[p]
 * are host float64 (dgamma_out/dbeta_out may be NULL only together); the call
 * synchronises `stream`.  zz_out as in qtn_contract. */
qtn_status qtn_energy_grad(qtn_net* net, qtn_mode mode, void* workspace, size_t ws_bytes, void* stream,
                           void* zz_out, double* energy_out, double* dgamma_out, double* dbeta_out);

/* Allocation-free variant of qtn_energy_grad, for callers that cannot
 * allocate device memory (code under graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  The workspace is the library's static
 * device scratch (QTN_SCRATCH_BYTES per GPU, reserved when the library's code
 * object is loaded on that GPU and held until the process ends); the caller
 * passes only the stream and the outputs, which mean what they mean for
 * qtn_energy_grad.  The sweep's kernels are launched directly on `stream` (the
 * batched form is not captured into a graph) and the call allocates nothing:
 * no hipMalloc, hipFree or allocating library routine.  Needs qtn_order and
 * qtn_set_params as usual.  QTN_ENOMEM when qtn_workspace_size(net, 1) exceeds
 * QTN_SCRATCH_BYTES (e.g. p >= 4 at tens of vertices).  Every call on one GPU
 * uses the same scratch, which keeps the last call's contents: calls that
 * overlap on one GPU (other threads, or streams not ordered with each other)
 * race and must be serialised by the caller.  qtn_edge_results with a NULL
 * workspace reads the per-edge results of such a call. */
#define QTN_SCRATCH_BYTES ((size_t)64 << 20)
qtn_status qtn_energy_grad_noalloc(qtn_net* net, qtn_mode mode, void* stream, void* zz_out, double* energy_out,
                                   double* dgamma_out, double* dbeta_out);

/* Per-edge results of the last sweep, host float64: zz[2*e] = Re <Z_j Z_k>,
 * zz[2*e+1] = Im; dzz (nullable) [n_edges][2p][2]: d<Z_j Z_k>/d(gamma_1..p,
 * beta_1..p), complex.  Reads the workspace of that sweep (`workspace` must be
 * the one it used, or NULL for "the last sweep's"); synchronises `stream` and
 * the sweep.  QTN_ESTATE before any sweep, or for dzz after a sweep without
 * the adjoint; QTN_EDEVICE when that sweep's persistent kernel reported an
 * error. */
qtn_status qtn_edge_results(qtn_net* net, const void* workspace, void* stream, double* zz, double* dzz);

qtn_status qtn_get_info(const qtn_net* net, qtn_info* out);

/* Census of the ordered plan's contraction steps (Section III.B: a step
 * multiplies the tensors holding its eliminated indices and sums those
 * indices) that contain a dense matrix product: two inputs A and B sharing at
 * least min_bits summed indices (the inner dimension K), each with at least
 * min_bits kept indices the other lacks (M and N); their shared kept indices
 * are batch dimensions.  n_steps: all steps; n_gemm: steps with such a pair;
 * gemm_flops / total_flops: real flops of those steps / of all steps (a step
 * of k inputs over union U: 6 (k - 1) 2^|U| for the products, plus the sums).
 * Host only; QTN_ESTATE before ordering. */
qtn_status qtn_gemm_census(const qtn_net* net, int32_t min_bits, int64_t* n_steps, int64_t* n_gemm,
                           double* gemm_flops, double* total_flops);
/* Per-cone statistics (host arrays of n_edges, each nullable): contraction
 * width, qubits in the light cone, tensor indices, leaf tensors, buckets,
 * algorithmic forward / adjoint bytes. */
qtn_status qtn_cone_stats(const qtn_net* net, int32_t* width, int32_t* n_qubits, int32_t* n_indices,
                          int32_t* n_tensors, int32_t* n_buckets, double* fwd_bytes, double* bwd_bytes);

/* Checks the plan's invariants (each index eliminated once, each bucket output
 * consumed exactly once by a later bucket that holds all its indices, masks
 * consistent with the union sets, widths, arena ranges disjoint and in bounds).
 * QTN_OK or QTN_EINVAL with the first violation in qtn_last_error(). */
qtn_status qtn_validate_plan(const qtn_net* net);

/* Memory admission and checkpointed adjoint: limit the workspace to about
 * `bytes` (0: no limit).  Every cone's leaf tables and their adjoints keep
 * their own place; the rest of each cone's working set (its dynamic region)
 * goes into a shared area: the batched sweep admits cones into it in queue
 * order, a cone waiting for the cones that last held its region.  A cone
 * whose dynamic region alone exceeds the area drops bucket outputs after the
 * forward sweep (largest first, where that shrinks the region) and the
 * adjoint sweep recomputes them right before their first use, after the
 * dropped outputs they read (results are unchanged; qtn_info reports the
 * recomputed outputs and their extra traffic).  QTN_ENOMEM (and no limit)
 * when even that cannot meet the budget.  Rebuilds and re-uploads the
 * device program. */
qtn_status qtn_set_memory_budget(qtn_net* net, size_t bytes);

/* Tile parameters; changing them rebuilds and re-uploads the device program. */
qtn_status qtn_get_tuning(const qtn_net* net, qtn_tuning* out);
qtn_status qtn_set_tuning(qtn_net* net, const qtn_tuning* t);

/* Project-written autotuner: times the batched sweep (with_grad as given) on
 * `stream` by coordinate descent over four groups (workgroup size and lane
 * cap; split thresholds seq_max_bits and tile_blocks; merge_bits and
 * merge_lam_bits; lds_threads and lds_kb), keeps the fastest setting and
 * returns it in *best (nullable).  Each candidate: one warm sweep, one timed
 * sweep, then the average of max(reps, about 25 ms worth, at most 200)
 * replays.  Needs qtn_set_params first and a workspace as for the sweep;
 * settings whose workspace would not fit in ws_bytes are skipped. */
qtn_status qtn_autotune(qtn_net* net, int32_t with_grad, void* workspace, size_t ws_bytes, void* stream,
                        int32_t reps, qtn_tuning* best);

/* Device time of the batched sweep's graph replay (leaf upload, queue reset,
 * persistent kernel, final reduction), summed over batched sweeps that wrote
 * host outputs since the last reset while sweep timing was on, from HIP events
 * recorded on the launch stream around the replay; and the number of such
 * sweeps. */
qtn_status qtn_kernel_time(qtn_net* net, double* ms_sum, int64_t* count, int32_t reset);

/* Sweep timing for qtn_kernel_time: with on != 0 every batched sweep records
 * a HIP event on its stream before and after the graph replay.  Off by
 * default: each event record adds several microseconds to a sweep of a few
 * hundred, and a synchronous caller waits for them.  Errors: QTN_EINVAL for a
 * NULL net. */
qtn_status qtn_set_sweep_timing(qtn_net* net, int32_t on);

/* Tile parameters of wide buckets by bucket signature band: band 0 = buckets
 * of more than seq_max_bits and at most 20 union bits, band 1 = 21..24, band 2
 * = 25 or more (Section III.B: the union of a bucket, its width + 1).  A field
 * of 0 keeps the global value, the qtn_tuning field of the same name; else
 * par_bits in 8..24, tile_blocks a power of two, loop_cap in 1..31.
 * Sequential programs (seq_max_bits or fewer union bits) are not affected. */
#define QTN_BANDS 3
typedef struct {
  int32_t par_bits, tile_blocks, loop_cap;
} qtn_band_tuning;
/* out[QTN_BANDS] (host). */
qtn_status qtn_get_band_tuning(const qtn_net* net, qtn_band_tuning* out);
/* in[QTN_BANDS] (host); rebuilds the device plan like qtn_set_tuning.
 * QTN_EINVAL for values out of range; a band setting that leaves some wide
 * bucket without a valid tiling is refused (QTN_EUNSUPPORTED) and the
 * previous bands are kept. */
qtn_status qtn_set_band_tuning(qtn_net* net, const qtn_band_tuning* in);
/* Per-band autotuner: for each band that holds a wide bucket, times the
 * band's ops as a sub-sweep of their own (as qtn_time_wide_sweep, all kinds,
 * `reps` replays) for par_bits in {19, 21, 23} x tile_blocks in {64, 128,
 * 256} with the bands already tuned in place, and keeps the fastest.  Leaves
 * the chosen bands set, writes them to best_out[QTN_BANDS] (nullable) and
 * the whole persistent sweep's time (as qtn_time_persistent) to ms_out
 * (nullable).  Workspace and errors as qtn_autotune; candidates whose plan
 * needs a larger workspace are skipped.  Host work: one plan rebuild per
 * candidate. */
qtn_status qtn_autotune_bands(qtn_net* net, int32_t with_grad, void* workspace, size_t ws_bytes, void* stream,
                              int32_t reps, qtn_band_tuning* best_out, double* ms_out);

/* Times the contraction ops of buckets whose output rank is >= min_width
 * (forward and, with with_grad, adjoint ops) one launch at a time on
 * `stream`, each replayed `reps` times between HIP events, reading the tensors
 * left in `workspace` by the last sweep of the same kind (atomic adjoint
 * outputs accumulate, so run a sweep again before reading results).  Returns
 * the algorithmic bytes of those ops (each input read once, output written
 * once; per replay) and their summed average device time. */
qtn_status qtn_time_wide_ops(qtn_net* net, int32_t with_grad, int32_t min_width, void* workspace, size_t ws_bytes,
                             void* stream, int32_t reps, double* bytes_out, double* ms_out, int64_t* n_ops_out);

/* In-sweep rate of the wide buckets: the contraction ops of buckets whose
 * output rank is in [min_width, max_width] (max_width <= 0: no upper bound)
 * and whose kind is in `kinds` (bit 0: forward contractions, bit 1: adjoint
 * ops that compute one input's adjoint, bit 2: fused adjoint ops; 0: all),
 * forward and, with with_grad, adjoint ops, as a queue of their own -- chained per light cone in program order, split into
 * the same tiles and list-scheduled as in the batched sweep -- run by one
 * launch of the persistent kernel, `reps` times (after one warm-up) between
 * HIP events on `stream`.  Reads the tensors left in `workspace` by the last
 * sweep of the same kind (outputs are overwritten or accumulated, so run a
 * sweep again before reading results).  Returns (each output nullable) the
 * algorithmic bytes of the selected contraction steps as qtn_info's fwd_bytes
 * and bwd_bytes count them (forward, if kinds has bit 0: every input read and
 * the output written; adjoint, if kinds has bit 1 or 2: the output adjoint
 * and every stored input read and every input adjoint written), the ops' own
 * operand bytes (each op's inputs read and output written once: one-input
 * adjoint passes read the output adjoint again), the average device time,
 * and the op and queue-item counts.  Allocates (and frees) the sub-queue's
 * device copy.  QTN_EDEVICE if a dependency wait gave up. */
qtn_status qtn_time_wide_sweep(qtn_net* net, int32_t with_grad, int32_t min_width, int32_t max_width, int32_t kinds,
                               void* workspace, size_t ws_bytes, void* stream, int32_t reps, double* bytes_out,
                               double* op_bytes_out, double* ms_out, int64_t* n_ops_out, int64_t* n_items_out);

/* Device time of the sweep's contraction kernels alone (the kernel of the
 * LDS-resident light cones, when there are any, then the persistent kernel
 * of the queued ones, when there are any): `reps` batched sweeps (after one
 * warm-up) are enqueued on `stream` without graph capture, each with HIP
 * events right before and after those kernels; *ms_out is their average.  Needs qtn_set_params and a workspace as for the sweep.  QTN_EDEVICE
 * if a sweep's dependency wait gave up. */
qtn_status qtn_time_persistent(qtn_net* net, int32_t with_grad, void* workspace, size_t ws_bytes, void* stream,
                               int32_t reps, double* ms_out);

/* Single-amplitude network (the paper's benchmark object, Section V):
 * <0...0|gamma beta> of the whole graph, ket only, with the same diagonal-gate
 * network rules (Sections III.A, IV.B) and a <0| leaf on the last index of
 * every qubit.  The net has one light cone (the whole graph); qtn_order /
 * qtn_order_rgreedy, qtn_set_params, qtn_set_tuning, qtn_workspace_size and
 * qtn_get_info apply as for qtn_build; read results with qtn_amplitude.
 * Arguments and errors as qtn_build (a graph with more than 4 connected
 * components is refused by the planner with QTN_EUNSUPPORTED). */
qtn_status qtn_build_amplitude(qtn_ctx* ctx, int32_t n_vertices, int32_t n_edges, const int32_t* edges, int32_t p,
                               qtn_dtype dtype, qtn_net** out);

/* Contracts an amplitude network: amp_out[0..1] = (re, im) of
 * <0...0|gamma beta> (host, float64).  With damp_out (host, [4p] doubles,
 * nullable) the adjoint sweep also runs and damp_out holds d amp / d gamma_l
 * (re, im) at 2l and d amp / d beta_l at 2p + 2l; the workspace must then be
 * sized with_grad = 1.  Synchronises `stream`.  QTN_ESTATE for a net made by
 * qtn_build. */
qtn_status qtn_amplitude(qtn_net* net, qtn_mode mode, void* workspace, size_t ws_bytes, void* stream,
                         double* amp_out, double* damp_out);

/* Cost model of the paper's comparison (Section IV; Figures diag_costs,
 * diag_costs_vs_n; Tables I and II), host only: the single-amplitude network
 * <0...0|gamma beta> of the graph built from the circuit in one of four ways
 * (default: CNOT / Z-rotation / H decomposition, every gate a full tensor with
 * fresh output indices; diagonal: gates keep the indices of the qubits they act
 * on diagonally, i.e. Z rotations and CNOT controls; ZZ: one two-qubit ZZ gate
 * per edge and one X rotation per qubit as full tensors; diagonal + ZZ: the ZZ
 * phase as a rank-2 tensor on the current indices), ordered by the library's
 * greedy or randomized greedy orderer (n_repeats, temperature, seed as in
 * qtn_order_rgreedy) and eliminated bucket by bucket.  Fills *out: index and
 * tensor counts, contraction width (largest intermediate rank), log2 of the
 * sum over buckets of 2^|union| (the FLOP estimate up to a constant) and the
 * ordering time.  QTN_EINVAL for bad arguments or graphs. */
typedef enum { QTN_NET_DEFAULT = 0, QTN_NET_DIAGONAL = 1, QTN_NET_ZZ = 2, QTN_NET_DIAGONAL_ZZ = 3 } qtn_net_variant;
typedef struct {
  int32_t n_indices, n_tensors;
  int32_t width;
  double log2_ops;
  double order_seconds;
} qtn_cost;
qtn_status qtn_cost_model(int32_t n_vertices, int32_t n_edges, const int32_t* edges, int32_t p,
                          qtn_net_variant variant, qtn_order_kind kind, int32_t n_repeats, double temperature,
                          uint64_t seed, qtn_cost* out);

/* qtn_cost_model that also writes the elimination order it evaluated into
 * order_out[0 .. out->n_indices) (host, caller-owned, order_cap entries).
 * Index ids follow the construction order: the initial index of every qubit
 * (qubit q gets id q), then each gate's new indices as the circuit creates
 * them (a two-qubit gate numbers its first qubit's new index first: the CNOT
 * control, the ZZ gate's first vertex of the edge as listed).  QTN_EINVAL as
 * qtn_cost_model, and when order_cap < n_indices (out is still filled). */
qtn_status qtn_cost_model_order(int32_t n_vertices, int32_t n_edges, const int32_t* edges, int32_t p,
                                qtn_net_variant variant, qtn_order_kind kind, int32_t n_repeats, double temperature,
                                uint64_t seed, qtn_cost* out, int32_t* order_out, int32_t order_cap);

/* Achievable-bandwidth reference: the library's plain copy kernel copies the
 * first half of the caller's device buffer `buf` (`bytes` long, 16-byte
 * aligned) onto its second half, `reps` times on `stream` after one warm-up,
 * between HIP events, for each of twelve launch shapes (1, 2 or 4 16-byte
 * loads in flight per thread; 4, 8, 16 or 32 workgroups of 256 threads per
 * compute unit).  *gbps_out = the best shape's (bytes read + bytes written)
 * per copy / average device time.  The buffer's contents are overwritten.  QTN_EINVAL for
 * a null buffer, fewer than 32 bytes or reps < 1. */
qtn_status qtn_copy_bandwidth(qtn_ctx* ctx, void* buf, size_t bytes, void* stream, int32_t reps, double* gbps_out);

void qtn_net_free(qtn_net* net);

#ifdef __cplusplus
}
#endif

#endif /* QTN_H */
