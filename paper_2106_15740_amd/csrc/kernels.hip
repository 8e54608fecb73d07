// HIP kernels for gfx950: bucket-elimination contraction of light-cone
// tensor networks (Section III.B of the paper: multiply every tensor holding
// the eliminated index over the union of their indices, then sum that index),
// its adjoint, the leaf-product tables of the diagonal-gate network
// (Section IV.B) and the final energy / gradient reductions.
//
// Every tensor stores its indices in elimination order, earliest index in the
// lowest bit, so the eliminated index of a bucket is bit 0 of every input that
// holds it: each thread loads the (x_v = 0, 1) pair of such an input with one
// 16-byte load and sums the pair in registers.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.hpp"

namespace qtn {

// ------------------------------------------------------------------ complex helpers
template <typename R>
struct CT;
template <>
struct CT<float> {
  using E = float2;
};
template <>
struct CT<double> {
  using E = double2;
};

template <typename E>
__device__ __forceinline__ E cmul(E a, E b) {
  E r;
  r.x = a.x * b.x - a.y * b.y;
  r.y = a.x * b.y + a.y * b.x;
  return r;
}
template <typename E>
__device__ __forceinline__ E cadd(E a, E b) {
  E r;
  r.x = a.x + b.x;
  r.y = a.y + b.y;
  return r;
}

__device__ __forceinline__ void load_pair(const float2* p, float2& a, float2& b) {
  float4 v = *reinterpret_cast<const float4*>(p);
  a = make_float2(v.x, v.y);
  b = make_float2(v.z, v.w);
}
__device__ __forceinline__ void load_pair(const double2* p, double2& a, double2& b) {
  a = p[0];
  b = p[1];
}
__device__ __forceinline__ void store_pair(float2* p, float2 a, float2 b) {
  *reinterpret_cast<float4*>(p) = make_float4(a.x, a.y, b.x, b.y);
}
__device__ __forceinline__ void store_pair(double2* p, double2 a, double2 b) {
  p[0] = a;
  p[1] = b;
}
__device__ __forceinline__ void atomic_add_c(float2* p, float2 v) {
  atomicAdd(&p->x, v.x);
  atomicAdd(&p->y, v.y);
}
__device__ __forceinline__ void atomic_add_c(double2* p, double2 v) {
  atomicAdd(&p->x, v.x);
  atomicAdd(&p->y, v.y);
}
__device__ __forceinline__ float2 shfl_xor_c(float2 v, int m) {
  return make_float2(__shfl_xor(v.x, m), __shfl_xor(v.y, m));
}
__device__ __forceinline__ double2 shfl_xor_c(double2 v, int m) {
  return make_double2(__shfl_xor(v.x, m), __shfl_xor(v.y, m));
}

// Element stride of union bit u inside a tensor whose union-bit mask is m.
__device__ __forceinline__ uint32_t bit_stride(uint32_t m, uint32_t u) {
  return ((m >> u) & 1u) ? (1u << __popc(m & ((1u << u) - 1u))) : 0u;
}

// ------------------------------------------------------------------ contraction op
// Runs the blocks [blk_begin, blk_end) of one OP_CONTRACT that fall to this
// workgroup.  A workgroup step covers nsub consecutive blocks (one per
// sub-block); the steps are cut into aligned power-of-two chunks, chunk
// wg_rank, wg_rank + wg_count, ... go to this workgroup, and each chunk is
// walked in Gray-code order so that consecutive steps differ in one block bit
// and every input offset moves by a single stride.  All threads take part in
// every step (tails are masked), so the LDS reduction may synchronise.

// Outputs per thread (2^nu) allowed for NIN inputs; the planner applies the
// same bound.
template <typename R, int NIN>
struct MaxU {
  static constexpr int value = (sizeof(R) == 4 && NIN <= 2) ? 2 : 1;
};

template <typename E>
struct RedBuf {
  E v[512 * 2];
};

template <typename R, int NIN, bool USE_LDS = false>
__device__ __forceinline__ void exec_contract(const OpDesc& d, typename CT<R>::E* __restrict__ arena, int64_t blk_begin,
                              int64_t blk_end, int64_t wg_rank, int64_t wg_count,
                              RedBuf<typename CT<R>::E>* __restrict__ red, typename CT<R>::E* lds = nullptr) {
  using E = typename CT<R>::E;
  constexpr int MAXU = MaxU<R, NIN>::value;
  const int tid = threadIdx.x;
  const int nl = d.nl, nu = d.nu, nk = d.nk;
  const int lanes = 1 << nl;
  const int sbits = 31 - __clz(blockDim.x >> nl);  // log2(sub-blocks per workgroup)
  const int sub = tid >> nl;
  const int lane = tid & (lanes - 1);
  const uint32_t out_mask = d.out_mask;
  const bool out_pair = out_mask & 1u;
  const bool atomic = d.flags & F_ATOMIC;
  const bool ldsred = d.flags & F_LDSRED;
  const int U = 1 << nu;

  uint32_t mask[NIN];
  uint32_t loff[NIN];
  const E* inp[NIN];
#pragma unroll
  for (int i = 0; i < NIN; ++i) {
    mask[i] = d.in_mask[i];
    if constexpr (USE_LDS)
      inp[i] = ((d.lds_mask >> i) & 1u) ? lds + d.lds_off[i] : arena + d.in_off[i];
    else
      inp[i] = arena + d.in_off[i];
    // lane offset: the strides of the lane bits are distinct powers of two
    uint32_t o = 0;
#pragma unroll
    for (int j = 0; j < MAXLANE; ++j) {
      const uint32_t sh = d.lsh[i][j];
      if (j < nl && sh != LSH_NONE) o |= ((uint32_t)(lane >> j) & 1u) << sh;
    }
    loff[i] = o;
  }
  uint32_t lout = 0;
#pragma unroll
  for (int j = 0; j < MAXLANE; ++j) {
    const uint32_t sh = d.lsh[MAXIN][j];
    if (j < nl && sh != LSH_NONE) lout |= ((uint32_t)(lane >> j) & 1u) << sh;
  }
  uint32_t us0[NIN];
#pragma unroll
  for (int i = 0; i < NIN; ++i) us0[i] = (MAXU > 1 && nu > 0) ? bit_stride(mask[i], d.zbit[nl]) : 0u;
  const uint32_t uo0 = (MAXU > 1 && nu > 0) ? bit_stride(out_mask, d.zbit[nl]) : 0u;
  E* outp;
  if constexpr (USE_LDS)
    outp = ((d.lds_mask >> MAXIN) & 1u) ? lds + d.lds_off[MAXIN] : arena + d.out_off;
  else
    outp = arena + d.out_off;
  const uint32_t lane_sum = d.lane_sum;
  const int zk0 = nl + nu;
  const int zb0 = nl + nu + nk;
  const int nb = d.nb;
  const int64_t nloop = int64_t(1) << nk;

  // workgroup steps and chunks: the block range (2^nb blocks, or an aligned
  // power-of-two tile of them) and wg_count are powers of two
  const int32_t nblk = (int32_t)(blk_end - blk_begin);
  const int lg_nblk = 31 - __clz(nblk);
  const int lg_st = lg_nblk > sbits ? lg_nblk - sbits : 0;
  const int lg_wg = 31 - __clz((uint32_t)wg_count);
  const int lg_chunk = lg_st > lg_wg ? lg_st - lg_wg : 0;
  const int64_t chunk = int64_t(1) << lg_chunk;
  const int64_t steps = int64_t(1) << lg_st;
  const int64_t nchunks = steps >> lg_chunk;

#pragma unroll 1
  for (int64_t ch = wg_rank; ch < nchunks; ch += wg_count) {
    const int64_t q0 = ch << lg_chunk;
    int64_t blk = blk_begin + (q0 << sbits) + sub;
    bool valid = blk < blk_end;
    uint32_t boff[NIN];
#pragma unroll
    for (int i = 0; i < NIN; ++i) boff[i] = loff[i];
    uint32_t bout = lout;
    {
      const int64_t b = valid ? blk : blk_begin;
      if (b) {
        for (int j = 0; j < nb; ++j)
          if ((b >> j) & 1) {
            const uint32_t u = d.zbit[zb0 + j];
#pragma unroll
            for (int i = 0; i < NIN; ++i) boff[i] += bit_stride(mask[i], u);
            bout += bit_stride(out_mask, u);
          }
      }
    }
#pragma unroll 1
    for (int64_t c = 0; c < chunk; ++c) {
      if (c) {
        // Gray step: block bit sbits + t flips
        const int t = __ffsll((unsigned long long)c) - 1;
        const int64_t g = c ^ (c >> 1);
        const bool up = (g >> t) & 1;
        const uint32_t u = d.zbit[zb0 + sbits + t];
#pragma unroll
        for (int i = 0; i < NIN; ++i) {
          const uint32_t st = bit_stride(mask[i], u);
          boff[i] = up ? boff[i] + st : boff[i] - st;
        }
        const uint32_t so = bit_stride(out_mask, u);
        bout = up ? bout + so : bout - so;
        blk = blk_begin + ((q0 + g) << sbits) + sub;
        valid = blk < blk_end;
      }
      if (q0 + c >= steps) break;  // uniform
      E acc0[MAXU], acc1[MAXU];
#pragma unroll
      for (int k = 0; k < MAXU; ++k) {
        acc0[k] = E{0, 0};
        acc1[k] = E{0, 0};
      }
      uint32_t koff[NIN];
#pragma unroll
      for (int i = 0; i < NIN; ++i) koff[i] = valid ? boff[i] : loff[i];
      uint32_t gray = 0;
#pragma unroll 1
      for (int64_t it = 0; it < nloop; ++it) {
        if (it) {
          const int fb = __ffsll((unsigned long long)it) - 1;  // Gray code over the summed loop bits
          const uint32_t u = d.zbit[zk0 + fb];
          gray ^= 1u << fb;
          const bool up = (gray >> fb) & 1u;
#pragma unroll
          for (int i = 0; i < NIN; ++i) {
            const uint32_t st = bit_stride(mask[i], u);
            koff[i] = up ? koff[i] + st : koff[i] - st;
          }
        }
#pragma unroll
        for (int k = 0; k < MAXU; ++k) {
          if (k < U) {
            E p0, p1;
#pragma unroll
            for (int i = 0; i < NIN; ++i) {
              const uint32_t o = koff[i] + (k ? us0[i] : 0u);
              E a0, a1;
              if (mask[i] & 1u) {
                load_pair(inp[i] + o, a0, a1);
              } else {
                a0 = inp[i][o];
                a1 = a0;
              }
              if (i == 0) {
                p0 = a0;
                p1 = a1;
              } else {
                p0 = cmul(p0, a0);
                p1 = cmul(p1, a1);
              }
            }
            acc0[k] = cadd(acc0[k], p0);
            acc1[k] = cadd(acc1[k], p1);
          }
        }
      }
#pragma unroll
      for (int k = 0; k < MAXU; ++k) {
        if (k < U) {  // uniform
          E s0 = acc0[k], s1 = acc1[k];
          if (!out_pair) s0 = cadd(s0, s1);
          if (lane_sum & 63u) {
            for (int j = 0; j < 6; ++j)
              if ((lane_sum >> j) & 1) {
                s0 = cadd(s0, shfl_xor_c(s0, 1 << j));
                if (out_pair) s1 = cadd(s1, shfl_xor_c(s1, 1 << j));
              }
          }
          if (ldsred) {
            // lanes of the same sub-block in other wavefronts: combine in LDS
            __syncthreads();
            red->v[2 * tid] = s0;
            red->v[2 * tid + 1] = s1;
            __syncthreads();
            const uint32_t hi = lane_sum & ~63u;
            if ((lane & hi) == 0)
              for (uint32_t m = hi; m; m = (m - 1) & hi) {
                s0 = cadd(s0, red->v[2 * (tid ^ (int)m)]);
                s1 = cadd(s1, red->v[2 * (tid ^ (int)m) + 1]);
              }
          }
          if (valid && (lane & lane_sum) == 0) {
            const uint32_t o = bout + (k ? uo0 : 0u);
            if (out_pair) {
              if (atomic) {
                atomic_add_c(outp + o, s0);
                atomic_add_c(outp + o + 1, s1);
              } else {
                store_pair(outp + o, s0, s1);
              }
            } else {
              if (atomic)
                atomic_add_c(outp + o, s0);
              else
                outp[o] = s0;
            }
          }
        }
      }
    }
  }
}

// ------------------------------------------------------------------ wide ops
// Executor of the ops flagged F_WIDE (buckets too wide for one workgroup).
// Everything that decides the instruction stream is a template parameter, so
// the step body has no branches between its loads: NIN inputs, S0 = 1 when
// input 0 lacks the eliminated index (the output adjoint of an adjoint op;
// every other input holds it and is loaded as a 16-byte pair), UU = 2^nu
// outputs per thread.  All loads of a step are issued before the first use.
// When the op has more per-thread output bits than UU covers (nu > log2 UU,
// at most one more), the step repeats for the extra bit.  KS: the UU slots
// hold the first log2 UU bits of the summation loop instead of outputs (ops
// with nu = 0 and nk >= log2 UU), so reductions keep as many loads in flight
// as element-wise ops and add the slots before the store.  The block range
// [blk_begin, blk_end) is an aligned power of two of at least one block per
// sub-block; offsets fit 32 bits (tensor rank <= 30).
template <typename R, int NIN, int S0, int UU, bool KS = false>
__device__ __forceinline__ void exec_wide(const OpDesc& d, typename CT<R>::E* __restrict__ arena, int64_t blk_begin,
                                          int64_t blk_end, int64_t wg_rank, int64_t wg_count,
                                          RedBuf<typename CT<R>::E>* __restrict__ red) {
  using E = typename CT<R>::E;
  const int tid = threadIdx.x;
  const int nl = d.nl, nk = d.nk;
  const int sbits = 31 - __clz(blockDim.x >> nl);
  const int sub = tid >> nl;
  const int lane = tid & ((1 << nl) - 1);
  const uint32_t out_mask = d.out_mask;
  const bool out_pair = out_mask & 1u;
  const bool atomic = d.flags & F_ATOMIC;
  const bool ldsred = d.flags & F_LDSRED;
  const uint32_t lane_sum = d.lane_sum;
  uint32_t mask[NIN], loff[NIN];
  const E* inp[NIN];
#pragma unroll
  for (int i = 0; i < NIN; ++i) {
    mask[i] = d.in_mask[i];
    inp[i] = arena + d.in_off[i];
    uint32_t o = 0;
#pragma unroll
    for (int j = 0; j < MAXLANE; ++j) {
      const uint32_t sh = d.lsh[i][j];
      if (j < nl && sh != LSH_NONE) o |= ((uint32_t)(lane >> j) & 1u) << sh;
    }
    loff[i] = o;
  }
  uint32_t lout = 0;
#pragma unroll
  for (int j = 0; j < MAXLANE; ++j) {
    const uint32_t sh = d.lsh[MAXIN][j];
    if (j < nl && sh != LSH_NONE) lout |= ((uint32_t)(lane >> j) & 1u) << sh;
  }
  // offsets of the UU slots of a thread: output bits zbit[nl], zbit[nl + 1],
  // or with KS the first loop bits (summed, so their output stride is 0)
  constexpr int LGU = UU == 4 ? 2 : (UU == 2 ? 1 : 0);
  const int zs = KS ? nl + d.nu : nl;
  uint32_t us[NIN][UU], uo[UU];
#pragma unroll
  for (int i = 0; i <= NIN; ++i) {
    const uint32_t m = i < NIN ? mask[i] : out_mask;
    const uint32_t s0 = UU > 1 ? bit_stride(m, d.zbit[zs]) : 0u;
    const uint32_t s1 = UU > 2 ? bit_stride(m, d.zbit[zs + 1]) : 0u;
#pragma unroll
    for (int k = 0; k < UU; ++k) {
      const uint32_t v = ((k & 1) ? s0 : 0u) + ((k & 2) ? s1 : 0u);
      if (i < NIN)
        us[i][k] = v;
      else
        uo[k] = v;
    }
  }
  E* outp = arena + d.out_off;
  constexpr int NU = KS ? 0 : LGU;
  const int nrep = d.nu > NU ? 2 : 1;
  uint32_t rs[NIN], rso = 0;  // strides of the repeated output bit
#pragma unroll
  for (int i = 0; i < NIN; ++i) rs[i] = nrep > 1 ? bit_stride(mask[i], d.zbit[nl + NU]) : 0u;
  if (nrep > 1) rso = bit_stride(out_mask, d.zbit[nl + NU]);
  const int zk0 = nl + d.nu + (KS ? LGU : 0), zb0 = nl + d.nu + nk;
  const int nloop = 1 << (KS ? nk - LGU : nk);
  const uint32_t base_blk = (uint32_t)blk_begin;
  const int lg_nblk = 31 - __clz((uint32_t)(blk_end - blk_begin));
  const int lg_st = lg_nblk - sbits;
  const int lg_wg = 31 - __clz((uint32_t)wg_count);
  const int lg_chunk = lg_st > lg_wg ? lg_st - lg_wg : 0;
  const int chunk = 1 << lg_chunk;
  const int nchunks = 1 << (lg_st - lg_chunk);
#pragma unroll 1
  for (int ch = (int)wg_rank; ch < nchunks; ch += (int)wg_count) {
    const uint32_t q0 = (uint32_t)ch << lg_chunk;
    const uint32_t blk = base_blk + (q0 << sbits) + (uint32_t)sub;
    uint32_t boff[NIN], bout = lout;
#pragma unroll
    for (int i = 0; i < NIN; ++i) boff[i] = loff[i];
    for (int j = 0; j < d.nb; ++j)
      if ((blk >> j) & 1u) {
        const uint32_t u = d.zbit[zb0 + j];
#pragma unroll
        for (int i = 0; i < NIN; ++i) boff[i] += bit_stride(mask[i], u);
        bout += bit_stride(out_mask, u);
      }
    // partial sums carried across block steps that flip only summed bits
    E acc0[UU], acc1[UU];
#pragma unroll
    for (int k = 0; k < UU; ++k) {
      acc0[k] = E{0, 0};
      acc1[k] = E{0, 0};
    }
#pragma unroll 1
    for (int c = 0; c < chunk; ++c) {
      if (c) {
        // Gray step: block bit sbits + t flips
        const int t = __ffs(c) - 1;
        const bool up = ((c ^ (c >> 1)) >> t) & 1;
        const uint32_t u = d.zbit[zb0 + sbits + t];
#pragma unroll
        for (int i = 0; i < NIN; ++i) {
          const uint32_t st = bit_stride(mask[i], u);
          boff[i] = up ? boff[i] + st : boff[i] - st;
        }
        const uint32_t so = bit_stride(out_mask, u);
        bout = up ? bout + so : bout - so;
      }
      // keep accumulating when the next step of this chunk flips a summed
      // bit (same outputs); nrep > 1 never has summed block bits
      const bool carry = nrep == 1 && c + 1 < chunk &&
                         bit_stride(out_mask, d.zbit[zb0 + sbits + __ffs(c + 1) - 1]) == 0u;
#pragma unroll 1
      for (int rep = 0; rep < nrep; ++rep) {
      uint32_t koff[NIN];
#pragma unroll
      for (int i = 0; i < NIN; ++i) koff[i] = boff[i] + (rep ? rs[i] : 0u);
      const uint32_t rout = bout + (rep ? rso : 0u);
      uint32_t gray = 0;
#pragma unroll 1
      for (int it = 0; it < nloop; ++it) {
        if (it) {
          const int fb = __ffs(it) - 1;  // Gray code over the summed loop bits
          const uint32_t u = d.zbit[zk0 + fb];
          gray ^= 1u << fb;
          const bool up = (gray >> fb) & 1u;
#pragma unroll
          for (int i = 0; i < NIN; ++i) {
            const uint32_t st = bit_stride(mask[i], u);
            koff[i] = up ? koff[i] + st : koff[i] - st;
          }
        }
        E a0[UU][NIN], a1[UU][NIN];
#pragma unroll
        for (int k = 0; k < UU; ++k)
#pragma unroll
          for (int i = 0; i < NIN; ++i) {
            const uint32_t o = koff[i] + us[i][k];
            if (i == 0 && S0 == 1)
              a0[k][i] = inp[i][o];
            else
              load_pair(inp[i] + o, a0[k][i], a1[k][i]);
          }
#pragma unroll
        for (int k = 0; k < UU; ++k) {
          E p0 = a0[k][0];
          E p1 = S0 == 1 ? a0[k][0] : a1[k][0];
#pragma unroll
          for (int i = 1; i < NIN; ++i) {
            p0 = cmul(p0, a0[k][i]);
            p1 = cmul(p1, a1[k][i]);
          }
          acc0[k] = cadd(acc0[k], p0);
          acc1[k] = cadd(acc1[k], p1);
        }
      }
      if (carry) continue;  // uniform
      if (KS) {
#pragma unroll
        for (int k = 1; k < UU; ++k) {
          acc0[0] = cadd(acc0[0], acc0[k]);
          acc1[0] = cadd(acc1[0], acc1[k]);
          acc0[k] = E{0, 0};
          acc1[k] = E{0, 0};
        }
      }
#pragma unroll
      for (int k = 0; k < (KS ? 1 : UU); ++k) {
        E s0 = acc0[k], s1 = acc1[k];
        acc0[k] = E{0, 0};
        acc1[k] = E{0, 0};
        if (!out_pair) s0 = cadd(s0, s1);
        if (lane_sum & 63u) {
          for (int j = 0; j < 6; ++j)
            if ((lane_sum >> j) & 1) {
              s0 = cadd(s0, shfl_xor_c(s0, 1 << j));
              if (out_pair) s1 = cadd(s1, shfl_xor_c(s1, 1 << j));
            }
        }
        if (ldsred) {
          // lanes of the same sub-block in other wavefronts: combine in LDS
          __syncthreads();
          red->v[2 * tid] = s0;
          red->v[2 * tid + 1] = s1;
          __syncthreads();
          const uint32_t hi = lane_sum & ~63u;
          if ((lane & hi) == 0)
            for (uint32_t m = hi; m; m = (m - 1) & hi) {
              s0 = cadd(s0, red->v[2 * (tid ^ (int)m)]);
              s1 = cadd(s1, red->v[2 * (tid ^ (int)m) + 1]);
            }
        }
        if ((lane & lane_sum) == 0) {
          const uint32_t o = rout + uo[k];
          if (out_pair) {
            if (atomic) {
              atomic_add_c(outp + o, s0);
              atomic_add_c(outp + o + 1, s1);
            } else {
              store_pair(outp + o, s0, s1);
            }
          } else {
            if (atomic)
              atomic_add_c(outp + o, s0);
            else
              outp[o] = s0;
          }
        }
      }
      }
    }
  }
}

// Largest per-thread output count of the wide executor for element type R:
// its own launches, and inside the persistent kernel (whose other state
// competes for registers; the rest of the op's output bits repeat the step).
template <typename R>
struct WideMaxU {
  static constexpr int value = sizeof(R) == 4 ? 4 : 2;
  static constexpr int in_persistent = sizeof(R) == 4 ? 2 : 1;
};

template <typename R, int NIN, int S0>
__device__ __forceinline__ void exec_wide_u(const OpDesc& d, typename CT<R>::E* arena, int64_t b0, int64_t b1,
                                            int64_t r, int64_t c, RedBuf<typename CT<R>::E>* red) {
  constexpr int M = WideMaxU<R>::in_persistent;
  if (M == 1 || (d.nu == 0 && d.nk == 0))
    exec_wide<R, NIN, S0, 1>(d, arena, b0, b1, r, c, red);
  else if (d.nu == 0 && d.nk >= (M == 4 ? 2 : 1))
    exec_wide<R, NIN, S0, M, true>(d, arena, b0, b1, r, c, red);
  else if (d.nu == 0)
    exec_wide<R, NIN, S0, 1>(d, arena, b0, b1, r, c, red);
  else
    exec_wide<R, NIN, S0, M>(d, arena, b0, b1, r, c, red);
}

template <typename R>
__device__ __forceinline__ void exec_wide_any(const OpDesc& d, typename CT<R>::E* arena, int64_t b0, int64_t b1,
                                              int64_t r, int64_t c, RedBuf<typename CT<R>::E>* red) {
  const bool s0 = !(d.in_mask[0] & 1u);
  switch (d.n_in * 2 + (s0 ? 1 : 0)) {
    case 2: exec_wide_u<R, 1, 0>(d, arena, b0, b1, r, c, red); break;
    case 3: exec_wide_u<R, 1, 1>(d, arena, b0, b1, r, c, red); break;
    case 4: exec_wide_u<R, 2, 0>(d, arena, b0, b1, r, c, red); break;
    case 5: exec_wide_u<R, 2, 1>(d, arena, b0, b1, r, c, red); break;
    case 6: exec_wide_u<R, 3, 0>(d, arena, b0, b1, r, c, red); break;
    case 7: exec_wide_u<R, 3, 1>(d, arena, b0, b1, r, c, red); break;
    case 8: exec_wide_u<R, 4, 0>(d, arena, b0, b1, r, c, red); break;
    default: exec_wide_u<R, 4, 1>(d, arena, b0, b1, r, c, red); break;
  }
}

// ------------------------------------------------------------------ fused adjoint
// Executor of OP_ADJOINT: every input adjoint of one wide bucket in one pass
// over its union, so the output adjoint and each input are read once.  Input
// 0 is the output adjoint (without bit 0), inputs 1..NIN-1 hold bit 0 and are
// loaded as pairs.  For each union element the adjoint of input i receives
// the output adjoint times the product of the other inputs, formed from
// prefix and suffix products.  An output that holds the loop bits gets one
// value per loop step: combined across the lanes it sums (shuffles; a
// sub-block is at most one wavefront) and stored.  Every other output sums
// the loop steps in registers and is written once per run of block steps
// that flip only bits it lacks: stored, or added with atomics into zeroed
// memory when it sums a block bit.  SL = 2: the first loop bit is unrolled
// into two slots whose loads are in flight together.  Block ranges as in
// exec_wide.
template <typename R, int NIN, int SL>
__device__ __forceinline__ void exec_adjoint(const OpDesc& d, typename CT<R>::E* __restrict__ arena, int64_t blk_begin,
                                             int64_t blk_end, int64_t wg_rank, int64_t wg_count) {
  using E = typename CT<R>::E;
  const int tid = threadIdx.x;
  const int nl = d.nl, nk = d.nk;
  const int sbits = 31 - __clz(blockDim.x >> nl);
  const int sub = tid >> nl;
  const int lane = tid & ((1 << nl) - 1);
  const int zk0 = nl + (SL > 1 ? 1 : 0), zb0 = nl + nk;
  uint32_t blockbits = 0;
  for (int z = zb0; z < d.nbits - 1; ++z) blockbits |= 1u << d.zbit[z];
  uint32_t mask[NIN], loff[NIN], lsum[NIN], ss[NIN];
  bool hold[NIN], atom[NIN];
  const E* inp[NIN];
  E* outp[NIN];
  uint32_t aheld = 0;  // bits held by an output that accumulates over the loop
#pragma unroll
  for (int i = 0; i < NIN; ++i) {
    mask[i] = d.in_mask[i];
    inp[i] = arena + d.in_off[i];
    outp[i] = arena + (i ? d.adj_off[i] : 0);
    hold[i] = i > 0 && nk > 0 && ((mask[i] >> d.zbit[nl]) & 1u);
    atom[i] = (blockbits & ~mask[i]) != 0;
    if (i > 0 && !hold[i]) aheld |= mask[i];
    uint32_t o = 0, ls = 0;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      const uint32_t sh = d.lsh[i][j];
      if (j < nl) {
        if (sh != LSH_NONE)
          o |= ((uint32_t)(lane >> j) & 1u) << sh;
        else
          ls |= 1u << j;
      }
    }
    loff[i] = o;
    lsum[i] = ls;
    ss[i] = SL > 1 ? bit_stride(mask[i], d.zbit[nl]) : 0u;
  }
  const int nloop = 1 << (nk - (SL > 1 ? 1 : 0));
  const uint32_t base_blk = (uint32_t)blk_begin;
  const int lg_nblk = 31 - __clz((uint32_t)(blk_end - blk_begin));
  const int lg_st = lg_nblk - sbits;
  const int lg_wg = 31 - __clz((uint32_t)wg_count);
  const int lg_chunk = lg_st > lg_wg ? lg_st - lg_wg : 0;
  const int chunk = 1 << lg_chunk;
  const int nchunks = 1 << (lg_st - lg_chunk);
  // combine a pair across the lanes in ls, then store or add it
  auto put = [&](E* p, E s0, E s1, uint32_t ls, bool at) {
    for (int j = 0; j < 6; ++j)
      if ((ls >> j) & 1u) {
        s0 = cadd(s0, shfl_xor_c(s0, 1 << j));
        s1 = cadd(s1, shfl_xor_c(s1, 1 << j));
      }
    if ((lane & ls) == 0) {
      if (at) {
        atomic_add_c(p, s0);
        atomic_add_c(p + 1, s1);
      } else {
        store_pair(p, s0, s1);
      }
    }
  };
#pragma unroll 1
  for (int ch = (int)wg_rank; ch < nchunks; ch += (int)wg_count) {
    const uint32_t q0 = (uint32_t)ch << lg_chunk;
    const uint32_t blk = base_blk + (q0 << sbits) + (uint32_t)sub;
    uint32_t boff[NIN];
#pragma unroll
    for (int i = 0; i < NIN; ++i) boff[i] = loff[i];
    for (int j = 0; j < d.nb; ++j)
      if ((blk >> j) & 1u) {
        const uint32_t u = d.zbit[zb0 + j];
#pragma unroll
        for (int i = 0; i < NIN; ++i) boff[i] += bit_stride(mask[i], u);
      }
    E acc0[NIN], acc1[NIN];
#pragma unroll
    for (int i = 0; i < NIN; ++i) {
      acc0[i] = E{0, 0};
      acc1[i] = E{0, 0};
    }
#pragma unroll 1
    for (int c = 0; c < chunk; ++c) {
      if (c) {
        const int t = __ffs(c) - 1;
        const bool up = ((c ^ (c >> 1)) >> t) & 1;
        const uint32_t u = d.zbit[zb0 + sbits + t];
#pragma unroll
        for (int i = 0; i < NIN; ++i) {
          const uint32_t st = bit_stride(mask[i], u);
          boff[i] = up ? boff[i] + st : boff[i] - st;
        }
      }
      // an accumulating output keeps its sums while the next step flips a bit
      // it does not hold
      const uint32_t nxt = c + 1 < chunk ? 1u << d.zbit[zb0 + sbits + __ffs(c + 1) - 1] : 0u;
      uint32_t koff[NIN];
#pragma unroll
      for (int i = 0; i < NIN; ++i) koff[i] = boff[i];
      uint32_t gray = 0;
#pragma unroll 1
      for (int it = 0; it < nloop; ++it) {
        if (it) {
          const int fb = __ffs(it) - 1;
          const uint32_t u = d.zbit[zk0 + fb];
          gray ^= 1u << fb;
          const bool up = (gray >> fb) & 1u;
#pragma unroll
          for (int i = 0; i < NIN; ++i) {
            const uint32_t st = bit_stride(mask[i], u);
            koff[i] = up ? koff[i] + st : koff[i] - st;
          }
        }
        E ob[SL], a0[SL][NIN], a1[SL][NIN];
#pragma unroll
        for (int s = 0; s < SL; ++s) {
          ob[s] = inp[0][koff[0] + (s ? ss[0] : 0u)];
#pragma unroll
          for (int i = 1; i < NIN; ++i) load_pair(inp[i] + koff[i] + (s ? ss[i] : 0u), a0[s][i], a1[s][i]);
        }
#pragma unroll
        for (int s = 0; s < SL; ++s) {
          E ex0[NIN], ex1[NIN];
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            // prefix products pr[i] = ob * x[1] ... x[i-1]; ex[i] = pr[i] * suffix
            E pr[NIN];
            pr[1] = ob[s];
#pragma unroll
            for (int i = 1; i + 1 < NIN; ++i) pr[i + 1] = cmul(pr[i], h ? a1[s][i] : a0[s][i]);
            E suf = E{1, 0};
#pragma unroll
            for (int i = NIN - 1; i >= 1; --i) {
              const E x = h ? a1[s][i] : a0[s][i];
              const E e = i == NIN - 1 ? pr[i] : cmul(pr[i], suf);
              suf = i == NIN - 1 ? x : cmul(x, suf);
              if (h)
                ex1[i] = e;
              else
                ex0[i] = e;
            }
          }
#pragma unroll
          for (int i = 1; i < NIN; ++i) {
            if (hold[i]) {
              put(outp[i] + koff[i] + (s ? ss[i] : 0u), ex0[i], ex1[i], lsum[i], atom[i]);
            } else {
              acc0[i] = cadd(acc0[i], ex0[i]);
              acc1[i] = cadd(acc1[i], ex1[i]);
            }
          }
        }
      }
      if (nxt && !(aheld & nxt)) continue;  // uniform: every accumulating output carries
#pragma unroll
      for (int i = 1; i < NIN; ++i) {
        if (hold[i] || (nxt && !(mask[i] & nxt))) continue;
        put(outp[i] + boff[i], acc0[i], acc1[i], lsum[i], atom[i]);
        acc0[i] = E{0, 0};
        acc1[i] = E{0, 0};
      }
    }
  }
}

__device__ __forceinline__ void lds_add(float2* p, float2 v) {
  atomicAdd(&p->x, v.x);
  atomicAdd(&p->y, v.y);
}
__device__ __forceinline__ void lds_add(double2* p, double2 v) {
  atomicAdd(&p->x, v.x);
  atomicAdd(&p->y, v.y);
}

// Executor of OP_ADJOINT ops flagged F_TILE: every input adjoint of a bucket
// whose inputs each lack part of the union, summed tile by tile in LDS.  A
// block is a tile; the workgroup's threads are its lanes (nl = log2 of the
// workgroup size) and walk the remaining tile bits in a per-thread loop.  Per
// union element, each output's value is combined across the lanes of the
// wavefront that it sums (shuffles) and added into its tile sum in LDS
// (2^(tile bits it holds) pairs, at lds + its base); at the end of the tile
// the sums are stored, or added with atomics when the output sums a block bit.
template <typename R, int NIN>
__device__ __forceinline__ void exec_tile(const OpDesc& d, typename CT<R>::E* __restrict__ arena, int64_t blk_begin,
                                          int64_t blk_end, int64_t wg_rank, int64_t wg_count,
                                          typename CT<R>::E* __restrict__ lds) {
  using E = typename CT<R>::E;
  const int tid = threadIdx.x;
  const int nl = d.nl, nk = d.nk, nb = d.nb;
  const int lane = tid & 63;
  uint32_t tmask = 0, blockbits = 0;
  for (int z = 0; z < nl + nk; ++z) tmask |= 1u << d.zbit[z];
  for (int z = nl + nk; z < d.nbits - 1; ++z) blockbits |= 1u << d.zbit[z];
  uint32_t mask[NIN], tm[NIN], loff[NIN], lidx[NIN], lsum[NIN], lbase[NIN];
  bool atom[NIN];
  const E* inp[NIN];
  E* outp[NIN];
  uint32_t total = 0;
#pragma unroll
  for (int i = 0; i < NIN; ++i) {
    mask[i] = d.in_mask[i];
    tm[i] = tmask & mask[i];
    inp[i] = arena + d.in_off[i];
    outp[i] = arena + (i ? d.adj_off[i] : 0);
    atom[i] = (blockbits & ~mask[i]) != 0;
    uint32_t o = 0, li = 0, ls = 0;
    for (int j = 0; j < nl; ++j) {
      const uint32_t u = d.zbit[j];
      const uint32_t bit = (uint32_t)(tid >> j) & 1u;
      if ((mask[i] >> u) & 1u) {
        o += bit * bit_stride(mask[i], u);
        li += bit * bit_stride(tm[i], u);
      } else if (j < 6) {
        ls |= 1u << j;
      }
    }
    loff[i] = o;
    lidx[i] = li;
    lsum[i] = ls;
    lbase[i] = total;
    if (i > 0) total += 2u << __popc(tm[i]);
  }
  const int nloop = 1 << nk;
  const uint32_t base_blk = (uint32_t)blk_begin;
  const int lg_nblk = 31 - __clz((uint32_t)(blk_end - blk_begin));
  const int lg_wg = 31 - __clz((uint32_t)wg_count);
  const int lg_chunk = lg_nblk > lg_wg ? lg_nblk - lg_wg : 0;
  const int chunk = 1 << lg_chunk;
  const int nchunks = 1 << (lg_nblk - lg_chunk);
#pragma unroll 1
  for (int ch = (int)wg_rank; ch < nchunks; ch += (int)wg_count) {
    const uint32_t blk0 = base_blk + ((uint32_t)ch << lg_chunk);
#pragma unroll 1
    for (int c = 0; c < chunk; ++c) {
      const uint32_t blk = blk0 + (uint32_t)c;
      uint32_t bb[NIN];  // block part of every operand's offset
#pragma unroll
      for (int i = 0; i < NIN; ++i) bb[i] = 0;
      for (int j = 0; j < nb; ++j)
        if ((blk >> j) & 1u) {
          const uint32_t u = d.zbit[nl + nk + j];
#pragma unroll
          for (int i = 0; i < NIN; ++i) bb[i] += bit_stride(mask[i], u);
        }
      for (uint32_t e = tid; e < total; e += blockDim.x) lds[e] = E{0, 0};
      __syncthreads();
      uint32_t koff[NIN], kl[NIN];
#pragma unroll
      for (int i = 0; i < NIN; ++i) {
        koff[i] = bb[i] + loff[i];
        kl[i] = lidx[i];
      }
      uint32_t gray = 0;
#pragma unroll 1
      for (int it = 0; it < nloop; ++it) {
        if (it) {
          const int fb = __ffs(it) - 1;
          const uint32_t u = d.zbit[nl + fb];
          gray ^= 1u << fb;
          const bool up = (gray >> fb) & 1u;
#pragma unroll
          for (int i = 0; i < NIN; ++i) {
            const uint32_t st = bit_stride(mask[i], u), sl = bit_stride(tm[i], u);
            koff[i] = up ? koff[i] + st : koff[i] - st;
            kl[i] = up ? kl[i] + sl : kl[i] - sl;
          }
        }
        E ob, a0[NIN], a1[NIN];
        ob = inp[0][koff[0]];
#pragma unroll
        for (int i = 1; i < NIN; ++i) load_pair(inp[i] + koff[i], a0[i], a1[i]);
        E ex0[NIN], ex1[NIN];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          E pr[NIN];
          pr[1] = ob;
#pragma unroll
          for (int i = 1; i + 1 < NIN; ++i) pr[i + 1] = cmul(pr[i], h ? a1[i] : a0[i]);
          E suf = E{1, 0};
#pragma unroll
          for (int i = NIN - 1; i >= 1; --i) {
            const E x = h ? a1[i] : a0[i];
            const E e = i == NIN - 1 ? pr[i] : cmul(pr[i], suf);
            suf = i == NIN - 1 ? x : cmul(x, suf);
            if (h)
              ex1[i] = e;
            else
              ex0[i] = e;
          }
        }
#pragma unroll
        for (int i = 1; i < NIN; ++i) {
          E s0 = ex0[i], s1 = ex1[i];
          for (int j = 0; j < 6; ++j)
            if ((lsum[i] >> j) & 1u) {
              s0 = cadd(s0, shfl_xor_c(s0, 1 << j));
              s1 = cadd(s1, shfl_xor_c(s1, 1 << j));
            }
          if ((lane & lsum[i]) == 0) {
            lds_add(lds + lbase[i] + 2 * kl[i], s0);
            lds_add(lds + lbase[i] + 2 * kl[i] + 1, s1);
          }
        }
      }
      __syncthreads();
      // the tile's sums: element e of output i holds its tile bits in order
#pragma unroll
      for (int i = 1; i < NIN; ++i) {
        const uint32_t n = 1u << __popc(tm[i]);
        for (uint32_t e = tid; e < n; e += blockDim.x) {
          uint32_t off = bb[i], rest = tm[i], k = e;
          while (rest) {
            const uint32_t u = __ffs(rest) - 1;
            rest &= rest - 1;
            if (k & 1u) off += bit_stride(mask[i], u);
            k >>= 1;
          }
          const E v0 = lds[lbase[i] + 2 * e], v1 = lds[lbase[i] + 2 * e + 1];
          if (atom[i]) {
            atomic_add_c(outp[i] + off, v0);
            atomic_add_c(outp[i] + off + 1, v1);
          } else {
            store_pair(outp[i] + off, v0, v1);
          }
        }
      }
      __syncthreads();
    }
  }
}

template <typename R>
__device__ __forceinline__ void exec_adjoint_any(const OpDesc& d, typename CT<R>::E* arena, int64_t b0, int64_t b1,
                                                 int64_t r, int64_t c, typename CT<R>::E* lds) {
  if (d.flags & F_TILE) {
    if (d.n_in == 3)
      exec_tile<R, 3>(d, arena, b0, b1, r, c, lds);
    else if (d.n_in == 4)
      exec_tile<R, 4>(d, arena, b0, b1, r, c, lds);
    return;
  }
  constexpr bool two = WideMaxU<R>::in_persistent > 1;
  const bool sl = two && d.nk >= 1;
  switch (d.n_in * 2 + (sl ? 1 : 0)) {
    case 6: exec_adjoint<R, 3, 1>(d, arena, b0, b1, r, c); break;
    case 7: exec_adjoint<R, 3, two ? 2 : 1>(d, arena, b0, b1, r, c); break;
    case 8: exec_adjoint<R, 4, 1>(d, arena, b0, b1, r, c); break;
    case 9: exec_adjoint<R, 4, two ? 2 : 1>(d, arena, b0, b1, r, c); break;
    default: break;
  }
}

template <typename R, int MAXNIN, bool USE_LDS>
__device__ __forceinline__ void exec_contract_any(const OpDesc& d, typename CT<R>::E* arena, int64_t b0, int64_t b1,
                                                  int64_t r, int64_t c, RedBuf<typename CT<R>::E>* red,
                                                  typename CT<R>::E* lds) {
  switch (d.n_in) {
    case 1: exec_contract<R, 1, USE_LDS>(d, arena, b0, b1, r, c, red, lds); break;
    case 2: exec_contract<R, 2, USE_LDS>(d, arena, b0, b1, r, c, red, lds); break;
    case 3: exec_contract<R, 3, USE_LDS>(d, arena, b0, b1, r, c, red, lds); break;
    case 4: if constexpr (MAXNIN >= 4) exec_contract<R, 4, USE_LDS>(d, arena, b0, b1, r, c, red, lds); break;
    case 5: if constexpr (MAXNIN >= 5) exec_contract<R, 5, USE_LDS>(d, arena, b0, b1, r, c, red, lds); break;
    case 6: if constexpr (MAXNIN >= 6) exec_contract<R, 6, USE_LDS>(d, arena, b0, b1, r, c, red, lds); break;
    case 7: if constexpr (MAXNIN >= 7) exec_contract<R, 7, USE_LDS>(d, arena, b0, b1, r, c, red, lds); break;
    default: if constexpr (MAXNIN >= 8) exec_contract<R, 8, USE_LDS>(d, arena, b0, b1, r, c, red, lds); break;
  }
}

// ------------------------------------------------------------------ leaf tables
// Leaf-product table of one bucket: entry e = prod over the bucket's leaves of
// leaf[e restricted to the leaf's indices].
template <typename R>
__device__ __forceinline__ void exec_leaf(const OpDesc& d, typename CT<R>::E* arena, const Env& env, int64_t wg_rank,
                          int64_t wg_count) {
  using E = typename CT<R>::E;
  const E* vals = reinterpret_cast<const E*>(env.leafvals);
  const int64_t n = int64_t(1) << d.nbits;
  E* out = arena + d.out_off;
  for (int64_t e = wg_rank * blockDim.x + threadIdx.x; e < n; e += wg_count * blockDim.x) {
    E p = {1, 0};
    for (int r = 0; r < d.aux1; ++r) {
      const LeafRef L = env.leafrefs[d.aux0 + r];
      int idx = (e >> L.pa) & 1;
      if (L.pb >= 0) idx |= ((e >> L.pb) & 1) << 1;
      p = cmul(p, vals[L.kind * 4 + idx]);
    }
    out[e] = p;
  }
}

// Parameter slot of a leaf kind inside a cone's result record: gamma_l at
// 2 + 2l, beta_l at 2 + 2p + 2l (real, imaginary); -1 for |+>, Z and <0|.
__device__ __forceinline__ int theta_slot(int kind, int p) {
  if (kind < 2 || kind >= 2 + 4 * p) return -1;
  const int l = (kind - 2) >> 2, t = (kind - 2) & 3;
  return t < 2 ? 2 + 2 * l : 2 + 2 * p + 2 * l;
}

template <typename R>
__device__ double2 block_sum(double2 v) {
  __shared__ double2 red[32];
  for (int m = 32; m >= 1; m >>= 1) {
    v.x += __shfl_xor(v.x, m);
    v.y += __shfl_xor(v.y, m);
  }
  const int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double2 s = make_double2(0, 0);
  if (threadIdx.x == 0)
    for (int i = 0; i < nw; ++i) {
      s.x += red[i].x;
      s.y += red[i].y;
    }
  return s;  // valid in thread 0
}

// dR/dtheta += sum_e Lbar[e] * d(leaf product)/dtheta [e], split per leaf:
// the derivative of one leaf times the product of the others.
template <typename R>
__device__ __forceinline__ void exec_leafgrad(const OpDesc& d, typename CT<R>::E* arena, const Env& env) {
  using E = typename CT<R>::E;
  const E* vals = reinterpret_cast<const E*>(env.leafvals);
  const E* dvals = reinterpret_cast<const E*>(env.dleafvals);
  const int64_t n = int64_t(1) << d.nbits;
  const E* lbar = arena + d.in_off[0];
  double* res = env.res + (int64_t)d.cone * env.res_stride;
  for (int r = 0; r < d.aux1; ++r) {
    const LeafRef L = env.leafrefs[d.aux0 + r];
    const int slot = theta_slot(L.kind, env.p);
    if (slot < 0) continue;  // uniform across the workgroup
    double2 acc = make_double2(0, 0);
    for (int64_t e = threadIdx.x; e < n; e += blockDim.x) {
      E t = lbar[e];
      for (int s = 0; s < d.aux1; ++s) {
        const LeafRef Ls = env.leafrefs[d.aux0 + s];
        int idx = (e >> Ls.pa) & 1;
        if (Ls.pb >= 0) idx |= ((e >> Ls.pb) & 1) << 1;
        t = cmul(t, s == r ? dvals[Ls.kind * 4 + idx] : vals[Ls.kind * 4 + idx]);
      }
      acc.x += (double)t.x;
      acc.y += (double)t.y;
    }
    const double2 s = block_sum<R>(acc);
    if (threadIdx.x == 0) {
      atomicAdd(res + slot, s.x);
      atomicAdd(res + slot + 1, s.y);
    }
  }
}

// Cone value R = product of the scalar outputs; with F_GRAD also the seed
// dR/dO_s = product of the other scalars, and zeroed gradient accumulators.
template <typename R>
__device__ __forceinline__ void exec_result(const OpDesc& d, typename CT<R>::E* arena, const Env& env,
                                            typename CT<R>::E* lds = nullptr) {
  using E = typename CT<R>::E;
  double* res = env.res + (int64_t)d.cone * env.res_stride;
  const int ns = d.n_in;
  auto at = [&](int i) -> E* {
    return (lds && ((d.lds_mask >> i) & 1u)) ? lds + d.lds_off[i] : arena + d.in_off[i];
  };
  if (threadIdx.x == 0) {
    double2 prod = make_double2(1, 0);
    for (int s = 0; s < ns; ++s) {
      const E x = *at(s);
      prod = cmul(prod, make_double2(x.x, x.y));
    }
    res[0] = prod.x;
    res[1] = prod.y;
  }
  if (d.flags & F_GRAD) {
    // seed of scalar s: product of the other scalars (thread s; no private arrays)
    for (int s = threadIdx.x; s < ns; s += blockDim.x) {
      double2 seed = make_double2(1, 0);
      for (int t = 0; t < ns; ++t)
        if (t != s) {
          const E x = *at(t);
          seed = cmul(seed, make_double2(x.x, x.y));
        }
      E o;
      o.x = (R)seed.x;
      o.y = (R)seed.y;
      *at(ns + s) = o;
    }
    for (int i = threadIdx.x; i < 4 * env.p; i += blockDim.x) res[2 + i] = 0.0;
  }
}

template <typename R>
__device__ __forceinline__ void exec_zero(const OpDesc& d, typename CT<R>::E* arena, int64_t wg_rank, int64_t wg_count) {
  using E = typename CT<R>::E;
  E* out = arena + d.out_off;
  const int64_t n = d.in_off[0];
  for (int64_t e = wg_rank * blockDim.x + threadIdx.x; e < n; e += wg_count * blockDim.x) out[e] = E{0, 0};
}

// MAXNIN < 0: contraction ops have exactly -MAXNIN inputs (plain launches are
// specialised per input count on the host); else up to MAXNIN inputs.
template <typename R, int MAXNIN, bool USE_LDS = false, bool WIDE = false>
__device__ __forceinline__ void exec_op(const OpDesc& d, const Env& env, int64_t b0, int64_t b1, int64_t wg_rank,
                                        int64_t wg_count, RedBuf<typename CT<R>::E>* red,
                                        typename CT<R>::E* lds = nullptr) {
  using E = typename CT<R>::E;
  E* arena = reinterpret_cast<E*>(env.arena);
  switch (d.kind) {
    case OP_CONTRACT:
      if constexpr (WIDE && !USE_LDS) {
        if (d.flags & F_WIDE) {
          exec_wide_any<R>(d, arena, b0, b1, wg_rank, wg_count, red);
          break;
        }
      }
      if constexpr (MAXNIN < 0)
        exec_contract<R, -MAXNIN>(d, arena, b0, b1, wg_rank, wg_count, red);
      else
        exec_contract_any<R, MAXNIN, USE_LDS>(d, arena, b0, b1, wg_rank, wg_count, red, lds);
      break;
    case OP_ADJOINT:
      if constexpr (WIDE && !USE_LDS) exec_adjoint_any<R>(d, arena, b0, b1, wg_rank, wg_count, lds);
      break;
    case OP_LEAF: exec_leaf<R>(d, arena, env, wg_rank, wg_count); break;
    case OP_RESULT:
      if (wg_rank == 0) exec_result<R>(d, arena, env, USE_LDS ? lds : nullptr);
      break;
    case OP_ZERO: exec_zero<R>(d, arena, wg_rank, wg_count); break;
    case OP_LEAFGRAD:
      if (wg_rank == 0) exec_leafgrad<R>(d, arena, env);
      break;
    default: break;
  }
}

// ------------------------------------------------------------------ kernels
// One op per launch (the plain per-edge loop).
// The descriptor is staged in LDS: the executors read its bit tables inside
// their loops, and an LDS read does not wait for the loads in flight.
__device__ __forceinline__ void stage_desc(OpDesc& sd, const OpDesc* ops, int op) {
  constexpr int W = sizeof(OpDesc) / sizeof(uint4);
  if (threadIdx.x < W) reinterpret_cast<uint4*>(&sd)[threadIdx.x] = reinterpret_cast<const uint4*>(ops + op)[threadIdx.x];
  __syncthreads();
}

// Workgroups are dispatched round-robin over the 8 XCDs: give each XCD a
// contiguous range of logical workgroups (and so of blocks), so blocks that
// share input data meet in the same L2.
__device__ __forceinline__ int64_t xcd_rank() {
  const int64_t G = gridDim.x;
  const int64_t w = blockIdx.x;
  return G % 8 == 0 ? (w % 8) * (G / 8) + w / 8 : w;
}

template <typename R, int NIN>
__global__ void __launch_bounds__(512) op_kernel(const OpDesc* __restrict__ ops, int op, Env env) {
  __shared__ RedBuf<typename CT<R>::E> red;
  __shared__ OpDesc d;
  stage_desc(d, ops, op);
  const int64_t nblocks = int64_t(1) << d.nb;
  exec_contract<R, NIN>(d, reinterpret_cast<typename CT<R>::E*>(env.arena), 0, nblocks, xcd_rank(), gridDim.x, &red);
}

// One F_WIDE op per launch, specialised like the executor.
template <typename R, int NIN, int S0, int UU, bool KS>
__global__ void __launch_bounds__(512) wide_kernel(const OpDesc* __restrict__ ops, int op, Env env) {
  __shared__ RedBuf<typename CT<R>::E> red;
  __shared__ OpDesc d;
  stage_desc(d, ops, op);
  const int64_t nblocks = int64_t(1) << d.nb;
  exec_wide<R, NIN, S0, UU, KS>(d, reinterpret_cast<typename CT<R>::E*>(env.arena), 0, nblocks, xcd_rank(), gridDim.x,
                            &red);
}

// One OP_ADJOINT op per launch.
template <typename R, int NIN, int SL>
__global__ void __launch_bounds__(512) adjoint_kernel(const OpDesc* __restrict__ ops, int op, Env env) {
  __shared__ OpDesc d;
  stage_desc(d, ops, op);
  const int64_t nblocks = int64_t(1) << d.nb;
  exec_adjoint<R, NIN, SL>(d, reinterpret_cast<typename CT<R>::E*>(env.arena), 0, nblocks, xcd_rank(), gridDim.x);
}

// One LDS-tiled OP_ADJOINT op per launch (dynamic LDS: the tile sums).
template <typename R, int NIN>
__global__ void __launch_bounds__(512) tile_kernel(const OpDesc* __restrict__ ops, int op, Env env) {
  __shared__ OpDesc d;
  extern __shared__ __align__(16) char tile_lds[];
  stage_desc(d, ops, op);
  const int64_t nblocks = int64_t(1) << d.nb;
  exec_tile<R, NIN>(d, reinterpret_cast<typename CT<R>::E*>(env.arena), 0, nblocks, xcd_rank(), gridDim.x,
                    reinterpret_cast<typename CT<R>::E*>(tile_lds));
}

// Leaf tables, results, zeroing and leaf gradients (one op per launch).
template <typename R>
__global__ void __launch_bounds__(512) misc_kernel(const OpDesc* __restrict__ ops, int op, Env env) {
  __shared__ RedBuf<typename CT<R>::E> red;
  const OpDesc& d = ops[op];
  exec_op<R, 1>(d, env, 0, 1, xcd_rank(), gridDim.x, &red);
}

constexpr int DESC_CHUNK = 16;

// Persistent sweep: workgroups pop items from a device queue in topological
// order; an item waits until its node counter is zero, runs, then releases
// its successor nodes.  Every item waits only on items earlier in the queue,
// which were already taken by running workgroups, so the sweep always drains.
// WIDE: the plan has F_WIDE ops (a separate instantiation keeps the register
// budget of narrow-only sweeps unchanged).
template <typename R, int MAXNIN, bool WIDE>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 4 : 1, 8))) persistent_kernel(const OpDesc* __restrict__ ops, const QItem* __restrict__ items,
                                                          int n_items, const int32_t* __restrict__ succ, int32_t* ctl,
                                                          Env env, long long spin_limit) {
  __shared__ RedBuf<typename CT<R>::E> red;
  __shared__ OpDesc sdesc[DESC_CHUNK];
  extern __shared__ __align__(16) char dyn_lds[];
  __shared__ int s_item;
  __shared__ int s_abort;
  int32_t* head = ctl;
  int32_t* err = ctl + 1;
  int32_t* node_cnt = ctl + 2;
  for (;;) {
    if (threadIdx.x == 0) {
      s_item = __hip_atomic_fetch_add(head, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      s_abort = 0;
    }
    __syncthreads();
    const int it = s_item;
    if (it >= n_items) break;
    const QItem I = items[it];
    if (threadIdx.x == 0 && I.node >= 0) {
      long long spins = 0;
      while (__hip_atomic_load(node_cnt + I.node, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) > 0) {
        __builtin_amdgcn_s_sleep(2);
        if (++spins > spin_limit) {
          __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          s_abort = 1;
          break;
        }
        if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
          s_abort = 1;
          break;
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
    if (!s_abort) {
      using E = typename CT<R>::E;
      E* lds = nullptr;
      if (I.copyin >= 0) {
        // LDS-resident cone: bring its leaf-product block into the LDS window
        const OpDesc& cp = ops[I.copyin];
        const E* src = reinterpret_cast<const E*>(env.arena) + cp.in_off[0];
        lds = reinterpret_cast<E*>(dyn_lds);
        for (int64_t t = threadIdx.x; t < cp.in_off[1]; t += blockDim.x) lds[t] = src[t];
        __syncthreads();
      }
      // descriptors are staged through LDS in chunks: one bulk copy instead of
      // a dependent global load per op
      for (int r = 0; r < 2; ++r) {
        const int lo = r ? I.op2_lo : I.op_lo;
        const int hi = r ? I.op2_hi : I.op_hi;
        for (int op0 = lo; op0 < hi; op0 += DESC_CHUNK) {
          const int nd = min(DESC_CHUNK, hi - op0);
          constexpr int W = sizeof(OpDesc) / sizeof(uint4);
          const uint4* src = reinterpret_cast<const uint4*>(ops + op0);
          uint4* dst = reinterpret_cast<uint4*>(sdesc);
          for (int t = threadIdx.x; t < nd * W; t += blockDim.x) dst[t] = src[t];
          __syncthreads();
          for (int j = 0; j < nd; ++j) {
            const OpDesc& d = sdesc[j];
            if (j > 0 && (d.flags & F_SYNC)) __syncthreads();
            const int64_t nblocks = (d.kind == OP_CONTRACT || d.kind == OP_ADJOINT) ? (int64_t(1) << d.nb) : 1;
            const int64_t b0 = I.blk_hi < 0 ? 0 : I.blk_lo;
            const int64_t b1 = I.blk_hi < 0 ? nblocks : I.blk_hi;
            if (lds)
              exec_op<R, MAXNIN, true>(d, env, b0, b1, 0, 1, &red, lds);
            else
              exec_op<R, MAXNIN, false, WIDE>(d, env, b0, b1, 0, 1, &red, reinterpret_cast<E*>(dyn_lds));
          }
          __syncthreads();
        }
      }
    }
    if (threadIdx.x == 0 && I.succ_hi > I.succ_lo) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      for (int s = I.succ_lo; s < I.succ_hi; ++s)
        __hip_atomic_fetch_add(node_cnt + succ[s], -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
  }
}

// Leaf-product tables (OP_LEAF) and leaf gradients (OP_LEAFGRAD) of every
// cone, one wavefront per op: the tables have a few to a few hundred entries,
// so a whole workgroup per op would idle.
__device__ __forceinline__ double wave_sum(double v) {
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
  return v;
}

constexpr int LG_MAXL = 16;  // leaves per table handled by the linear-time leaf gradient

template <typename R>
__global__ void __launch_bounds__(256) leaf_batch_kernel(const OpDesc* __restrict__ ops, int lo, int hi, Env env,
                                                         int32_t* ctl, const int32_t* __restrict__ ctl_init,
                                                         int n_nodes) {
  // with ctl: also reset the queue head, the error flag and the node
  // counters of the persistent sweep that follows
  if (ctl)
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_nodes + 2; i += gridDim.x * blockDim.x)
      ctl[i] = i < 2 ? 0 : ctl_init[i - 2];
  using E = typename CT<R>::E;
  const int lane = threadIdx.x & 63;
  const int wave = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  const int nwaves = (int)((gridDim.x * blockDim.x) >> 6);
  // the leaf values and their derivatives (4 entries per kind, 3 + 4p kinds,
  // p <= 16) are looked up once per leaf and table entry: keep them in LDS
  constexpr int NV = 4 * (3 + 4 * 16);
  __shared__ E s_vals[NV], s_dvals[NV];
  const int nv = 4 * (3 + 4 * env.p);
  for (int i = threadIdx.x; i < nv && i < NV; i += blockDim.x) {
    s_vals[i] = reinterpret_cast<const E*>(env.leafvals)[i];
    s_dvals[i] = reinterpret_cast<const E*>(env.dleafvals)[i];
  }
  __syncthreads();
  const E* vals = s_vals;
  const E* dvals = s_dvals;
  E* arena = reinterpret_cast<E*>(env.arena);
  for (int op = lo + wave; op < hi; op += nwaves) {
    const OpDesc& d = ops[op];
    const int64_t n = int64_t(1) << d.nbits;
    const LeafRef* refs = env.leafrefs + d.aux0;
    if (d.kind == OP_LEAF) {
      E* out = arena + d.out_off;
      for (int64_t e = lane; e < n; e += 64) {
        E pr = {1, 0};
        for (int r = 0; r < d.aux1; ++r) {
          const LeafRef L = refs[r];
          int idx = (e >> L.pa) & 1;
          if (L.pb >= 0) idx |= ((e >> L.pb) & 1) << 1;
          pr = cmul(pr, vals[L.kind * 4 + idx]);
        }
        out[e] = pr;
      }
    } else if (d.kind == OP_LEAFGRAD) {
      // dR/dtheta += sum_e Lbar[e] * (derivative of one leaf) * (the other
      // leaves).  Up to LG_MAXL leaves: per entry, suffix products of the
      // leaves, then one forward pass with the running prefix (3L complex
      // multiplies instead of L^2); leaves come sorted by angle, so one
      // atomic per angle.
      const E* lbar = arena + d.in_off[0];
      double* res = env.res + (int64_t)d.cone * env.res_stride;
      const int L = d.aux1;
      if (L <= LG_MAXL) {
        double ax[LG_MAXL], ay[LG_MAXL];
#pragma unroll
        for (int q = 0; q < LG_MAXL; ++q) ax[q] = ay[q] = 0.0;
        for (int64_t e = lane; e < n; e += 64) {
          E suf[LG_MAXL + 1];
          suf[LG_MAXL] = E{1, 0};
#pragma unroll
          for (int q = LG_MAXL - 1; q >= 0; --q) {
            if (q < L) {
              const LeafRef Lq = refs[q];
              int idx = (e >> Lq.pa) & 1;
              if (Lq.pb >= 0) idx |= ((e >> Lq.pb) & 1) << 1;
              suf[q] = cmul(vals[Lq.kind * 4 + idx], suf[q + 1]);
            } else {
              suf[q] = E{1, 0};
            }
          }
          E pre = lbar[e];
#pragma unroll
          for (int q = 0; q < LG_MAXL; ++q) {
            if (q < L) {
              const LeafRef Lq = refs[q];
              int idx = (e >> Lq.pa) & 1;
              if (Lq.pb >= 0) idx |= ((e >> Lq.pb) & 1) << 1;
              const E t = cmul(cmul(pre, dvals[Lq.kind * 4 + idx]), suf[q + 1]);
              ax[q] += (double)t.x;
              ay[q] += (double)t.y;
              pre = cmul(pre, vals[Lq.kind * 4 + idx]);
            }
          }
        }
        // per angle: sum the leaves in the lane, then across the wavefront
        int cur = -1;
        double sx = 0, sy = 0;
#pragma unroll
        for (int q = 0; q <= LG_MAXL; ++q) {
          const int slot = q < L ? theta_slot(refs[q].kind, env.p) : -2;  // uniform across the wavefront
          if (slot == -1) continue;
          if (slot != cur && cur >= 0) {
            const double wx = wave_sum(sx), wy = wave_sum(sy);
            if (lane == 0) {
              atomicAdd(res + cur, wx);
              atomicAdd(res + cur + 1, wy);
            }
          }
          if (slot == -2) break;
          if (slot != cur) {
            cur = slot;
            sx = sy = 0;
          }
          if (q < LG_MAXL) {
            sx += ax[q];
            sy += ay[q];
          }
        }
      } else {
        for (int r = 0; r < L; ++r) {
          const int slot = theta_slot(refs[r].kind, env.p);
          if (slot < 0) continue;  // uniform across the wavefront
          double ax = 0, ay = 0;
          for (int64_t e = lane; e < n; e += 64) {
            E t = lbar[e];
            for (int q = 0; q < L; ++q) {
              const LeafRef Ls = refs[q];
              int idx = (e >> Ls.pa) & 1;
              if (Ls.pb >= 0) idx |= ((e >> Ls.pb) & 1) << 1;
              t = cmul(t, q == r ? dvals[Ls.kind * 4 + idx] : vals[Ls.kind * 4 + idx]);
            }
            ax += (double)t.x;
            ay += (double)t.y;
          }
          ax = wave_sum(ax);
          ay = wave_sum(ay);
          if (lane == 0) {
            atomicAdd(res + slot, ax);
            atomicAdd(res + slot + 1, ay);
          }
        }
      }
    }
  }
}

// Copy of a few hundred bytes between device memory and mapped pinned host
// memory (leaf values in, results out): a kernel node keeps the sweep's
// graph free of copy-engine transfers and their start-up latency.
__global__ void __launch_bounds__(256) small_copy_kernel(const uint32_t* __restrict__ src, uint32_t* __restrict__ dst,
                                                         int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = src[i];
}

// Plain device copy (16-byte words, grid-stride): the achievable-bandwidth
// reference the contraction kernels are compared against.
__global__ void __launch_bounds__(256) copy_kernel(const uint4* __restrict__ src, uint4* __restrict__ dst, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

// Resets the queue head, the error flag and the node counters (a kernel, not
// a memset, so the sweep can be captured in a graph).
__global__ void reset_ctl_kernel(int32_t* ctl, const int32_t* __restrict__ init, int n_nodes) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_nodes + 2; i += gridDim.x * blockDim.x)
    ctl[i] = i < 2 ? 0 : init[i - 2];
}

// E = sum_c (1 - Re R_c)/2, dE/dtheta = -1/2 sum_c Re dR_c/dtheta, and the
// per-edge <Z_j Z_k> = R_c in the caller's dtype.
template <typename R>
__global__ void final_kernel(const double* __restrict__ res, int res_stride, int n_cones, int p, int with_grad,
                             typename CT<R>::E* zz_out, double* fin, double* host_fin, const int32_t* ctl,
                             int32_t* host_ctl) {
  using E = typename CT<R>::E;
  const int nv = 1 + (with_grad ? 2 * p : 0);
  for (int c = threadIdx.x; c < n_cones; c += blockDim.x)
    if (zz_out) {
      E z;
      z.x = (R)res[(int64_t)c * res_stride];
      z.y = (R)res[(int64_t)c * res_stride + 1];
      zz_out[c] = z;
    }
  for (int v = 0; v < nv; ++v) {
    double acc = 0;
    for (int c = threadIdx.x; c < n_cones; c += blockDim.x) {
      const double* r = res + (int64_t)c * res_stride;
      acc += v == 0 ? 0.5 * (1.0 - r[0]) : -0.5 * r[2 + 2 * (v - 1)];
    }
    const double2 s = block_sum<R>(make_double2(acc, 0));
    if (threadIdx.x == 0) {
      fin[v] = s.x;
      if (host_fin) host_fin[v] = s.x;
    }
    __syncthreads();
  }
  // the queue head and the persistent kernel's error flag, next to the results
  if (host_ctl && threadIdx.x < 2) host_ctl[threadIdx.x] = ctl ? ctl[threadIdx.x] : 0;
}

// ------------------------------------------------------------------ host launchers
template <typename R>
static hipError_t launch_op_t(const OpDesc* d_ops, const OpDesc& h, int op, const Env& env, int threads, int max_grid,
                              hipStream_t st) {
  int64_t grid = 1;
  if (h.kind == OP_CONTRACT || h.kind == OP_ADJOINT) {
    const int64_t nsub = threads >> h.nl;
    const int64_t nblocks = int64_t(1) << h.nb;
    grid = (nblocks + nsub - 1) / nsub;
    // partial sums that meet in atomics: each workgroup walks several block
    // steps (carrying its sums across them) instead of adding once per step
    if (h.flags & F_ATOMIC) grid = std::min<int64_t>(grid, 1024);
  } else if (h.kind == OP_LEAF) {
    grid = ((int64_t(1) << h.nbits) + threads - 1) / threads;
  } else if (h.kind == OP_ZERO) {
    grid = (h.in_off[0] + threads - 1) / threads;
  }
  if (grid > max_grid) grid = max_grid;
  if (grid < 1) grid = 1;
  // a power of two: the contraction executor splits its blocks by shifts
  grid = int64_t(1) << (63 - __builtin_clzll((unsigned long long)grid));
  const dim3 g((unsigned)grid), b(threads);
  if (h.kind == OP_ADJOINT && (h.flags & F_TILE)) {
    const size_t lb = (size_t)h.aux0 * sizeof(typename CT<R>::E);
    if (h.n_in == 3)
      hipLaunchKernelGGL((tile_kernel<R, 3>), g, b, lb, st, d_ops, op, env);
    else if (h.n_in == 4)
      hipLaunchKernelGGL((tile_kernel<R, 4>), g, b, lb, st, d_ops, op, env);
    else
      return hipErrorInvalidValue;
    return hipGetLastError();
  }
  if (h.kind == OP_ADJOINT) {
    const bool sl = h.nk >= 1;
    switch (h.n_in * 2 + (sl ? 1 : 0)) {
      case 6: hipLaunchKernelGGL((adjoint_kernel<R, 3, 1>), g, b, 0, st, d_ops, op, env); break;
      case 7: hipLaunchKernelGGL((adjoint_kernel<R, 3, 2>), g, b, 0, st, d_ops, op, env); break;
      case 8: hipLaunchKernelGGL((adjoint_kernel<R, 4, 1>), g, b, 0, st, d_ops, op, env); break;
      case 9: hipLaunchKernelGGL((adjoint_kernel<R, 4, 2>), g, b, 0, st, d_ops, op, env); break;
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  if (h.kind != OP_CONTRACT) {
    hipLaunchKernelGGL((misc_kernel<R>), g, b, 0, st, d_ops, op, env);
    return hipGetLastError();
  }
  if (h.flags & F_WIDE) {
    const bool s0 = !(h.in_mask[0] & 1u);
    const int uu = 1 << h.nu;
    // no output bits per thread: the slots take the first loop bits (one or two)
    const int ks = h.nu == 0 ? std::min(h.nk, WideMaxU<R>::value == 4 ? 2 : 1) : 0;
#define QTN_WIDE(N, S, UU, KS) hipLaunchKernelGGL((wide_kernel<R, N, S, UU, KS>), g, b, 0, st, d_ops, op, env)
#define QTN_WIDE_U(N, S)                              \
  do {                                                \
    if (ks == 1)                                      \
      QTN_WIDE(N, S, 2, true);                        \
    else if (ks == 2)                                 \
      QTN_WIDE(N, S, 4, true);                        \
    else if (uu == 1)                                 \
      QTN_WIDE(N, S, 1, false);                       \
    else if (uu == 2 || WideMaxU<R>::value < 4)       \
      QTN_WIDE(N, S, 2, false);                       \
    else                                              \
      QTN_WIDE(N, S, WideMaxU<R>::value, false);      \
  } while (0)
    switch (h.n_in * 2 + (s0 ? 1 : 0)) {
      case 2: QTN_WIDE_U(1, 0); break;
      case 3: QTN_WIDE_U(1, 1); break;
      case 4: QTN_WIDE_U(2, 0); break;
      case 5: QTN_WIDE_U(2, 1); break;
      case 6: QTN_WIDE_U(3, 0); break;
      case 7: QTN_WIDE_U(3, 1); break;
      case 8: QTN_WIDE_U(4, 0); break;
      case 9: QTN_WIDE_U(4, 1); break;
      default: return hipErrorInvalidValue;
    }
#undef QTN_WIDE_U
#undef QTN_WIDE
    return hipGetLastError();
  }
  switch (h.n_in) {
    case 1: hipLaunchKernelGGL((op_kernel<R, 1>), g, b, 0, st, d_ops, op, env); break;
    case 2: hipLaunchKernelGGL((op_kernel<R, 2>), g, b, 0, st, d_ops, op, env); break;
    case 3: hipLaunchKernelGGL((op_kernel<R, 3>), g, b, 0, st, d_ops, op, env); break;
    case 4: hipLaunchKernelGGL((op_kernel<R, 4>), g, b, 0, st, d_ops, op, env); break;
    case 5: hipLaunchKernelGGL((op_kernel<R, 5>), g, b, 0, st, d_ops, op, env); break;
    case 6: hipLaunchKernelGGL((op_kernel<R, 6>), g, b, 0, st, d_ops, op, env); break;
    case 7: hipLaunchKernelGGL((op_kernel<R, 7>), g, b, 0, st, d_ops, op, env); break;
    case 8: hipLaunchKernelGGL((op_kernel<R, 8>), g, b, 0, st, d_ops, op, env); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_op(bool c128, const OpDesc* d_ops, const OpDesc& h, int op, const Env& env, int threads,
                     int max_grid, hipStream_t st) {
  return c128 ? launch_op_t<double>(d_ops, h, op, env, threads, max_grid, st)
              : launch_op_t<float>(d_ops, h, op, env, threads, max_grid, st);
}

hipError_t launch_batch(bool c128, const OpDesc* d_ops, int lo, int hi, const Env& env, hipStream_t st, int32_t* ctl,
                        const int32_t* ctl_init, int n_nodes) {
  if (hi <= lo && !ctl) return hipSuccess;
  // 4 wavefronts per workgroup, one op each
  const int grid = std::max(1, std::min(std::max(hi - lo, 0) / 4 + 1, 4096));
  if (c128)
    hipLaunchKernelGGL(leaf_batch_kernel<double>, dim3(grid), dim3(256), 0, st, d_ops, lo, hi, env, ctl, ctl_init,
                       n_nodes);
  else
    hipLaunchKernelGGL(leaf_batch_kernel<float>, dim3(grid), dim3(256), 0, st, d_ops, lo, hi, env, ctl, ctl_init,
                       n_nodes);
  return hipGetLastError();
}

hipError_t launch_small_copy(const void* src, void* dst, size_t bytes, hipStream_t st) {
  if (bytes == 0) return hipSuccess;
  if (bytes % 4 || bytes > (size_t(1) << 20)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(small_copy_kernel, dim3(1), dim3(256), 0, st, reinterpret_cast<const uint32_t*>(src),
                     reinterpret_cast<uint32_t*>(dst), (int)(bytes / 4));
  return hipGetLastError();
}

hipError_t launch_copy(const void* src, void* dst, size_t n16, hipStream_t st) {
  if (n16 == 0) return hipSuccess;
  hipLaunchKernelGGL(copy_kernel, dim3(8192), dim3(256), 0, st, reinterpret_cast<const uint4*>(src),
                     reinterpret_cast<uint4*>(dst), n16);
  return hipGetLastError();
}

hipError_t launch_reset(int32_t* ctl, const int32_t* init, int n_nodes, hipStream_t st) {
  int grid = (n_nodes + 2 + 255) / 256;
  if (grid > 1024) grid = 1024;
  hipLaunchKernelGGL(reset_ctl_kernel, dim3(grid), dim3(256), 0, st, ctl, init, n_nodes);
  return hipGetLastError();
}

template <typename R, int M, bool W>
static hipError_t launch_persistent_m(const OpDesc* ops, const QItem* items, int n_items, const int32_t* succ,
                                      int32_t* ctl, const Env& env, int threads, int grid, size_t lds_bytes,
                                      long long spin_limit, hipStream_t st) {
  if (lds_bytes > 0) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&persistent_kernel<R, M, W>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((persistent_kernel<R, M, W>), dim3(grid), dim3(threads), lds_bytes, st, ops, items, n_items,
                     succ, ctl, env, spin_limit);
  return hipGetLastError();
}

template <typename R, bool W>
static hipError_t launch_persistent_t(int max_nin, const OpDesc* ops, const QItem* items, int n_items,
                                      const int32_t* succ, int32_t* ctl, const Env& env, int threads, int grid,
                                      size_t lds_bytes, long long spin_limit, hipStream_t st) {
  if (max_nin <= 3)
    return launch_persistent_m<R, 3, W>(ops, items, n_items, succ, ctl, env, threads, grid, lds_bytes, spin_limit, st);
  if (max_nin <= 5)
    return launch_persistent_m<R, 5, W>(ops, items, n_items, succ, ctl, env, threads, grid, lds_bytes, spin_limit, st);
  return launch_persistent_m<R, 8, W>(ops, items, n_items, succ, ctl, env, threads, grid, lds_bytes, spin_limit, st);
}

hipError_t launch_persistent(bool c128, bool wide, int max_nin, const OpDesc* ops, const QItem* items, int n_items,
                             const int32_t* succ, int32_t* ctl, const Env& env, int threads, int grid,
                             size_t lds_bytes, long long spin_limit, hipStream_t st) {
  if (c128)
    return wide ? launch_persistent_t<double, true>(max_nin, ops, items, n_items, succ, ctl, env, threads, grid,
                                                    lds_bytes, spin_limit, st)
                : launch_persistent_t<double, false>(max_nin, ops, items, n_items, succ, ctl, env, threads, grid,
                                                     lds_bytes, spin_limit, st);
  return wide ? launch_persistent_t<float, true>(max_nin, ops, items, n_items, succ, ctl, env, threads, grid, lds_bytes,
                                                 spin_limit, st)
              : launch_persistent_t<float, false>(max_nin, ops, items, n_items, succ, ctl, env, threads, grid,
                                                  lds_bytes, spin_limit, st);
}

hipError_t launch_final(bool c128, const double* res, int res_stride, int n_cones, int p, int with_grad, void* zz_out,
                        double* fin, double* host_fin, const int32_t* ctl, int32_t* host_ctl, hipStream_t st) {
  if (c128)
    hipLaunchKernelGGL(final_kernel<double>, dim3(1), dim3(256), 0, st, res, res_stride, n_cones, p, with_grad,
                       reinterpret_cast<double2*>(zz_out), fin, host_fin, ctl, host_ctl);
  else
    hipLaunchKernelGGL(final_kernel<float>, dim3(1), dim3(256), 0, st, res, res_stride, n_cones, p, with_grad,
                       reinterpret_cast<float2*>(zz_out), fin, host_fin, ctl, host_ctl);
  return hipGetLastError();
}

}  // namespace qtn
