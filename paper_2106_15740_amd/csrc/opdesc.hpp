// Plain-old-data records shared by the host planner and the HIP kernels.
#pragma once

#include <cstdint>

namespace qtn {

constexpr int MAXIN = 8;     // tensor inputs of one contraction op
constexpr int MAXBITS = 31;  // union bits of one bucket (output rank <= 30)
constexpr int MAXLANE = 10;  // lane bits of one op
constexpr uint8_t LSH_NONE = 0xff;

enum OpKind : int32_t {
  OP_CONTRACT = 0,  // out[pext(u,out)] (+)= sum over unmasked bits of prod_i in_i[pext(u,mask_i)]
  OP_LEAF = 1,      // leaf-product table of one bucket
  OP_RESULT = 2,    // cone value R = prod of scalar outputs; optional adjoint seeds
  OP_ZERO = 3,      // zero a range of the arena
  OP_LEAFGRAD = 4,  // dR/dtheta from the adjoint of one leaf-product table
  OP_ADJOINT = 6,   // every input adjoint of one wide bucket in one pass over its union (see adj_off)
};

enum OpFlags : int32_t {
  F_ATOMIC = 1,  // output receives partial sums from several blocks / waves
  F_GRAD = 2,    // OP_RESULT also writes adjoint seeds
  F_LDSRED = 4,  // summed lane bits >= 6: partial sums are combined across wavefronts in LDS
  F_SYNC = 8,    // in a sequential program: barrier before this op (it depends on an op since the last one)
  F_WIDE = 16,   // run by the wide-op executor: <= 4 inputs, inputs 1.. hold the eliminated index, every block
                 // range it is given holds at least one block per sub-block
  F_TILE = 32,   // OP_ADJOINT summed per tile in LDS: the workgroup's threads are the lanes, blocks are tiles,
                 // aux0 = LDS elements of the tile sums
  F_OUTER = 64,  // OP_ADJOINT whose outputs sum in 2^nu register slots per thread (nu slot bits after the
                 // lanes, then the loop bits); outputs holding the loop bits are flushed every loop step
};

// A contraction op iterates the union index u of a bucket.  Bit 0 of u is the
// eliminated index and is handled inside each thread as a pair (x_v = 0, 1).
// The other union bits are listed in zbit[] in iteration order: the first nl
// are lanes of a sub-block of 2^nl threads, the next nu are output bits
// unrolled inside a thread, the next nk are a per-thread summation loop, the
// last nb enumerate blocks.  Input i reads element pext(u, in_mask[i]) at
// in_off[i]; the output is written at pext(u, out_mask).  lane_sum marks the
// lane bits that are summed (reduced across lanes after the loop).
struct alignas(16) OpDesc {
  int32_t kind;
  int32_t n_in;
  int32_t nbits;      // union bits (contract) / table rank (leaf, leafgrad)
  int32_t nl, nu, nk, nb;
  int32_t flags;
  uint32_t out_mask;
  uint32_t lane_sum;  // lane z-bits that are summed (shuffles below bit 6, LDS above)
  int32_t cone;
  int32_t aux0, aux1;  // leaf ref range for OP_LEAF / OP_LEAFGRAD
  int64_t out_off;
  int64_t in_off[MAXIN];
  uint32_t in_mask[MAXIN];
  uint8_t zbit[32];
  // lane offsets without bit arithmetic on the device: for operand i (output:
  // MAXIN) and lane bit j < nl, the element stride is 1 << lsh[i][j], or 0
  // when lsh[i][j] == LSH_NONE
  uint8_t lsh[MAXIN + 1][MAXLANE];
  uint8_t pad_[6];
  // OP_ADJOINT: input 0 is the output adjoint (without the eliminated index,
  // bit 0), inputs 1.. hold bit 0; for every i with bit i of adj_sel set, the
  // adjoint of input i (same index set in_mask[i]) is written at adj_off[i]:
  // stored element by element when in_mask[i] holds every union bit, else
  // summed into zeroed memory with atomics.  out_off / out_mask are unused.
  int64_t adj_off[MAXIN];
  uint32_t adj_sel;
  uint32_t pad2_[3];
};
static_assert(sizeof(OpDesc) % 16 == 0, "OpDesc is copied in 16-byte words");
static_assert(sizeof(OpDesc) == 368, "OpDesc layout");

struct LeafRef {
  int16_t kind;
  int8_t pa, pb;  // bit positions inside the leaf-product table (pb < 0: rank 1)
};

// Compact op of an LDS-resident light-cone program (the batched sweep runs
// such a cone's whole program in one workgroup, every tensor in LDS).  The
// union bits of a contraction are renumbered as "dimensions": the output's
// bits first (in union order, so output element o is the first n_out
// dimensions read as a number), then the summed bits.  Input i reads element
// sum over set dimensions j of 2^shift_i[j], where shift_i[j] is nibble j of
// shift[i] (0xf: input i lacks dimension j).
enum SmallKind : uint8_t {
  S_CONTRACT = 0,  // out[o] = sum over summed dims of prod_i in_i[...]
  S_COPYIN = 1,    // copy aux1 elements of the arena from gout (the cone's leaf-product block) to LDS offset 0
  S_RESULT = 2,    // cone value R = prod of the n_in (<= 4) scalars at in_off[]; SF_GRAD: seeds at in_off[4 + s]
};
enum SmallFlags : uint8_t {
  SF_SYNC = 1,  // barrier before the op (it reads or overwrites data of an op since the last barrier)
  SF_SPLIT = 8,  // S_CONTRACT shared by every wavefront of the workgroup (each takes a chunk of its outputs)
  SF_GOUT = 2,  // the output goes to global memory at element offset gout (not LDS)
  SF_GRAD = 4,  // S_RESULT also writes the adjoint seeds and zeroes the gradient accumulators
};
struct alignas(16) SmallOp {  // the executor reads byte 0 (kind), 4 (flags) and 5 (wave) first
  uint8_t kind;
  uint8_t n_in;
  uint8_t nbits;   // contraction: union bits (<= 15)
  uint8_t n_out;   // contraction: output bits
  uint8_t flags;
  uint8_t wave;         // wavefront of the workgroup that runs the op (modulo the wavefronts present)
  uint8_t pad0[2];
  uint16_t out_off;     // LDS element offset of the output
  uint16_t in_off[8];   // LDS element offsets of the inputs (S_RESULT: scalars, then seeds)
  uint16_t pad1[3];
  uint64_t shift[8];    // per input: 16 nibbles, the element stride (log2) of each dimension
  int64_t gout;         // global element offset (SF_GOUT output; S_COPYIN source)
  int32_t aux0, aux1;   // S_COPYIN: aux1 = elements
  int32_t cone;
  int32_t pad2[3];
};
static_assert(sizeof(SmallOp) == 128, "SmallOp is copied in 16-byte words");

// Persistent-queue work item: ops [op_lo, op_hi) then [op2_lo, op2_hi) run
// in sequence by one workgroup over all their blocks (blk_hi < 0), or blocks
// [blk_lo, blk_hi) of the single op op_lo.  The item may start once
// node_cnt[node] reaches zero (node < 0: no dependency) and on completion
// decrements node_cnt[s] for every s in succ[succ_lo, succ_hi).
struct QItem {
  int32_t op_lo, op_hi;
  int32_t op2_lo, op2_hi;  // second range (-1: none)
  int32_t blk_lo, blk_hi;
  int32_t node;
  int32_t succ_lo, succ_hi;
  int32_t pad[3];
};

}  // namespace qtn
