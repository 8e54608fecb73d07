// Host-side planner: graph intake, per-edge light cone, diagonal-gate tensor
// network, greedy elimination order, bucket plan and the per-cone op program
// that the HIP kernels execute.  Nothing here touches the GPU.
#pragma once

#include <cstdint>
#include <functional>
#include <string>
#include <vector>

#include "opdesc.hpp"

namespace qtn {

// Leaf tensor kinds.  Every leaf has rank 1 or 2 and is one of 4p+3 distinct
// values: |+> (1,1)/sqrt2, the observable Z = (1,-1), per layer l the ket ZZ
// phase tensor, its conjugate (bra), the ket mixer exp(-i beta X) and its
// conjugate, and the projector <0| = (1,0) of single-amplitude networks.
enum LeafKind : int32_t { LK_PLUS = 0, LK_ZOBS = 1 };
inline int32_t lk_zz(int l) { return 2 + 4 * l + 0; }     // l is 0-based layer
inline int32_t lk_zzb(int l) { return 2 + 4 * l + 1; }
inline int32_t lk_mx(int l) { return 2 + 4 * l + 2; }
inline int32_t lk_mxb(int l) { return 2 + 4 * l + 3; }
inline int32_t lk_proj0(int p) { return 2 + 4 * p; }      // <0| on the last index of a qubit (amplitude networks)
inline int32_t n_leaf_kinds(int p) { return 3 + 4 * p; }

struct Leaf {
  int32_t kind;
  int32_t a, b;  // index ids; b = -1 for rank-1 leaves
};

// One contraction step.  A plain bucket eliminates one index (Section III.B);
// a merged bucket eliminates the indices of a connected piece of the
// elimination tree in one step (the union of its members' tensors, summed
// over all of their indices at once).  The eliminated indices are the lowest
// n_elim bits of the union.
struct Bucket {
  int32_t v = -1;                 // first eliminated index (bit 0)
  int32_t n_elim = 1;             // eliminated indices: union bits 0 .. n_elim-1
  std::vector<int32_t> uni;       // union, sorted by elimination position (uni[0] == v)
  std::vector<int32_t> in_bkt;    // producer bucket of each intermediate input
  std::vector<uint32_t> in_mask;  // its mask over union bits
  std::vector<int32_t> leaves;    // leaf ids absorbed by this bucket
  uint32_t lam_mask = 0;          // union bits carried by the leaf product (0: no leaves)
  int32_t consumer = -1;          // bucket that reads this output (-1: scalar result)
  int nbits() const { return (int)uni.size(); }
  int out_rank() const { return (int)uni.size() - n_elim; }
  uint32_t elim_mask() const { return (1u << n_elim) - 1u; }
  int lam_rank() const { return __builtin_popcount(lam_mask); }
};

// Logical buffers of a cone program.  While programs are built, an operand
// offset holds buf_code(kind, bucket) (a negative number); the arena layout
// replaces it by an absolute element offset.
enum BufKind : int32_t {
  BK_OUT = 0,     // forward output of a bucket
  BK_ADJ = 1,     // adjoint of that output
  BK_REC = 2,     // forward output recomputed during the adjoint sweep
  BK_LAM = 3,     // leaf-product table
  BK_LAMADJ = 4,  // adjoint of the leaf-product table
};
inline int64_t buf_code(int kind, int bucket) { return -((((int64_t)bucket) << 3 | kind) + 1); }
inline bool is_code(int64_t off) { return off < 0; }
inline int code_kind(int64_t code) { return (int)((-code - 1) & 7); }
inline int code_bucket(int64_t code) { return (int)((-code - 1) >> 3); }

// Lifetime and placement of one logical buffer in the cone's arena.
struct BufLife {
  int64_t code = 0;
  int64_t size = 0;
  int def = -1, last = -1;  // positions in the gradient program
  int64_t off = -1;         // element offset relative to the cone's base
};

// One edge term <Z_j Z_k>: the light-cone network and its contraction plan.
struct Cone {
  int32_t j = 0, k = 0;
  int32_t n_qubits = 0;
  int32_t n_idx = 0;
  std::vector<Leaf> leaves;
  std::vector<int32_t> order;     // elimination order (index ids)
  int32_t width = 0;              // largest bucket output rank
  std::vector<Bucket> plain;      // one bucket per index, in elimination order
  std::vector<Bucket> buckets;    // contraction steps (plain buckets, small ones merged), in order
  std::vector<int32_t> scalars;   // buckets whose output has rank 0
  // arena: [leaf tables][their adjoints][buffers placed by lifetime]
  std::vector<char> recompute;    // bucket outputs not kept for the adjoint sweep (recomputed there)
  std::vector<BufLife> bufs;      // placement of every logical buffer
  int64_t base = 0;               // element offset of the cone's pinned part (leaf tables, their adjoints)
  int64_t arena_elems = 0;        // elements the cone occupies (pinned part, then its dynamic region)
  int64_t dyn_start = 0;          // cone-relative offset where the dynamic region starts (= pinned elements)
  int64_t dyn_base = 0;           // offset of the dynamic region inside the plan's dynamic area
  int64_t keep_all_elems = 0;     // elements without any recomputation
  int64_t lam_base = 0, lam_size = 0;  // contiguous block of the leaf-product tables (absolute)
  double fwd_bytes_alg = 0, bwd_bytes_alg = 0, fwd_flops = 0, rec_bytes = 0;
};

struct TuneParams {
  int threads = 256;        // workgroup size of every kernel
  int lane_cap = 8;         // at most this many lane bits per op
  int seq_max_bits = 16;    // ops with more union bits run as multi-workgroup tiles
  int tile_blocks = 8;      // blocks of a wide op handled by one queue item
  int loop_cap = 12;        // summed bits kept inside a thread before spilling to atomics
  int unroll_cap = 1;       // output bits handled inside one thread of a wide op (<= 1)
  int par_bits = 21;        // a wide op aims at >= 2^par_bits threads
  int elem_bytes = 8;       // 8: complex64, 16: complex128 (set by build_programs)
  int lds_kb = 96;          // LDS window cap for LDS-resident cones (0: never)
  int merge_bits = 12;       // merge a bucket into its consumer while the merged union has <= this many bits (0: off)
  int merge_lam_bits = 7;   // ... and its leaf-product table has <= this many bits
  int lane_low = 1;         // wide ops: lanes on the lowest union bits (1) or the lowest output bits (0)
  int fuse_adjoint = 1;     // wide buckets: every input adjoint in one pass where a loop-bit group fits (1), also
                            // LDS tiles for the others (2), or one op per input (0)
  int lds_threads = 256;    // workgroup size of the kernel that runs the LDS-resident cones
  // Tile parameters of wide ops by union size (bucket signature bands: <= 20,
  // 21..24, >= 25 union bits); 0 keeps the value above.
  struct Band {
    int par_bits = 0, tile_blocks = 0, loop_cap = 0;
  };
  static constexpr int kBands = 3;
  Band band[kBands];
  static int band_of(int nbits) { return nbits <= 20 ? 0 : (nbits <= 24 ? 1 : 2); }
  // the parameters an op with nbits union bits is planned with
  TuneParams for_bits(int nbits) const {
    TuneParams t = *this;
    if (nbits <= seq_max_bits) return t;  // sequential programs keep the global values
    const Band& b = band[band_of(nbits)];
    if (b.par_bits) t.par_bits = b.par_bits;
    if (b.tile_blocks) t.tile_blocks = b.tile_blocks;
    if (b.loop_cap) t.loop_cap = b.loop_cap;
    return t;
  }
};

struct Plan {
  int32_t n = 0, p = 0;
  std::vector<std::pair<int32_t, int32_t>> edges;
  std::vector<Cone> cones;
  int order_kind = 0;
  bool ordered = false;
  TuneParams tune;
  // device programs
  std::vector<OpDesc> ops;          // all ops of all cones
  std::vector<int32_t> cone_fwd_lo, cone_fwd_hi, cone_adj_lo, cone_adj_hi;
  std::vector<LeafRef> leafrefs;
  int32_t leaf_lo = 0, leaf_hi = 0;    // all OP_LEAF ops (run before the sweep)
  int32_t lgrad_lo = 0, lgrad_hi = 0;  // all OP_LEAFGRAD ops (run after the adjoint sweep)
  int32_t lgrad_mid = 0;               // [lgrad_lo, lgrad_mid): tables of at most 8 leaves, then the others
  std::vector<char> cone_lds;          // cone runs LDS-resident in the persistent sweep (as a SmallOp program)
  std::vector<SmallOp> small;          // LDS-resident programs of those cones
  std::vector<int32_t> small_fwd_lo, small_fwd_hi;    // per cone: forward-only program in `small`
  std::vector<int32_t> small_grad_lo, small_grad_hi;  // per cone: forward + adjoint program
  int64_t lds_elems = 0;               // largest LDS window needed (elements)
  int64_t arena_fwd = 0, arena_grad = 0;  // elements needed without / with gradient
  int64_t mem_budget = 0;           // arena budget in elements (0: unlimited)
  int64_t dyn_off = 0;              // arena offset of the dynamic area (after every cone's pinned part)
  // under a budget: the cones each queued cone waits for (they last held part
  // of its dynamic region); empty without a budget
  std::vector<std::vector<int32_t>> cone_pred;
  int sched_workers = 1024;  // resident workgroups the queue order is scheduled for
  // persistent-queue items (forward-only and forward+gradient programs)
  std::vector<QItem> items_fwd, items_grad;
  std::vector<int32_t> node_init_fwd, node_init_grad;   // initial dependency counts
  std::vector<int32_t> succ_fwd, succ_grad;             // successor node lists (CSR payload)
  // LDS-resident cones: (lo, hi) ranges into `small`, one per cone, longest first
  std::vector<int32_t> small_items_fwd, small_items_grad;
  int32_t max_width = 0;
};

// Returns "" on success, else an error message.
std::string validate_graph(int32_t n, int32_t m, const int32_t* edges, int32_t p);
void build_cones(Plan& P);
// Single-amplitude network <0...0|gamma beta> of the whole graph (ket only):
// one "cone" whose result is the amplitude.
void build_amplitude(Plan& P);
struct OrderOptions {
  int kind = 0;              // 0 = min-degree, 1 = min-fill
  int repeats = 0;           // randomized runs on top of the deterministic one
  double temperature = 0.0;  // Boltzmann temperature of the randomized choice
  uint64_t seed = 0;
};
void order_cones(Plan& P, const OrderOptions& O, int n_threads);

// Contraction cost of the single-amplitude network under one of the paper's
// four constructions (0 default, 1 diagonal, 2 ZZ gates, 3 diagonal + ZZ),
// ordered by the same greedy / randomized greedy orderer.  order_out
// (nullable) receives the elimination order (index ids in construction order).
struct CostEstimate {
  int n_indices = 0, n_tensors = 0;
  int width = 0;          // largest intermediate rank
  double log2_ops = 0;    // log2 of sum over buckets of 2^|union|
};
CostEstimate cost_model(int n, const std::vector<std::pair<int32_t, int32_t>>& edges, int p, int variant,
                        const OrderOptions& O, std::vector<int>* order_out = nullptr);
// Builds every cone's forward and adjoint programs, places the buffers by
// lifetime (recomputing bucket outputs in the adjoint sweep where the memory
// budget requires it) and resolves all operand offsets.
std::string build_programs(Plan& P, int elem_bytes);
// Persistent-queue items for the forward (grad = false) or forward + adjoint
// program; items are in topological order.  Cones that run LDS-resident are
// not in the queue: they get one (lo, hi) range each in small_items_*.
void build_items(Plan& P, bool grad);
// The same queue construction into q; with `keep`, only the ops it accepts
// (chained per cone in program order, never LDS-resident): a sub-sweep for
// measurement.
struct Queue {
  std::vector<QItem> items;
  std::vector<int32_t> init, succ;
};
void build_queue(const Plan& P, bool grad, const std::function<bool(int32_t)>& keep, Queue& q);
// Plan invariants; "" if all hold, else the first violation.
std::string validate_plan(const Plan& P);

}  // namespace qtn
