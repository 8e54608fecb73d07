// Device executors of the contraction, adjoint and leaf ops (shared by the
// per-op kernels and the persistent sweep; every kernel translation unit
// includes this header and instantiates only its own kernels).
#pragma once

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

// v of lane + 2^J (lanes whose bit J is 0 only: those read inside their row of
// 16, where J < 4 is a row shift of the VALU's data-parallel lane moves, no
// LDS round trip; the others read an unspecified value)
template <int J>
__device__ __forceinline__ float lane_down(float v) {
  if constexpr (J < 4)
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x100 | (1 << J), 0xf, 0xf, true));
  else
    return __shfl_xor(v, 1 << J);
}
template <int J>
__device__ __forceinline__ double lane_down(double v) {
  if constexpr (J < 4) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x100 | (1 << J), 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x100 | (1 << J), 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
  } else {
    return __shfl_xor(v, 1 << J);
  }
}
template <int J, typename C>
__device__ __forceinline__ C lane_down_c(C v) {
  C r;
  r.x = lane_down<J>(v.x);
  r.y = lane_down<J>(v.y);
  return r;
}

// Parameter slot of a leaf kind inside a cone's result record: gamma_l at
// 2 + 2l, beta_l at 2 + 2p + 2l (real, imaginary); -1 for |+>, Z and <0|.
__device__ __forceinline__ int theta_slot(int kind, int p) {
  if (kind < 2 || kind >= 2 + 4 * p) return -1;
  const int l = (kind - 2) >> 2, t = (kind - 2) & 3;
  return t < 2 ? 2 + 2 * l : 2 + 2 * p + 2 * l;
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
  return v;
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

template <typename R, int NIN>
__device__ __forceinline__ void exec_contract(const OpDesc& d, typename CT<R>::E* __restrict__ arena, int64_t blk_begin,
                              int64_t blk_end, int64_t wg_rank, int64_t wg_count,
                              RedBuf<typename CT<R>::E>* __restrict__ red) {
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
  E* outp = arena + d.out_off;
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
// the step body has no branches between its loads: NIN inputs, of which the
// first S0 (0, 1 or 2) lack the eliminated index and are loaded as single
// elements (the output adjoint of an adjoint op; an input of a merged step
// that a later bucket brought in), every other input holds it and is loaded
// as a 16-byte pair, UU = 2^nu
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
            if (i < S0)
              a0[k][i] = inp[i][o];
            else
              load_pair(inp[i] + o, a0[k][i], a1[k][i]);
          }
#pragma unroll
        for (int k = 0; k < UU; ++k) {
          E p0 = a0[k][0];
          E p1 = S0 >= 1 ? a0[k][0] : a1[k][0];
#pragma unroll
          for (int i = 1; i < NIN; ++i) {
            p0 = cmul(p0, a0[k][i]);
            p1 = cmul(p1, i < S0 ? a0[k][i] : a1[k][i]);
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
  // leading inputs without the eliminated index (the planner puts them first)
  const int ns = !(d.in_mask[0] & 1u) ? (d.n_in > 1 && !(d.in_mask[1] & 1u) ? 2 : 1) : 0;
  switch (d.n_in * 3 + ns) {
    case 3: exec_wide_u<R, 1, 0>(d, arena, b0, b1, r, c, red); break;
    case 4: exec_wide_u<R, 1, 1>(d, arena, b0, b1, r, c, red); break;
    case 6: exec_wide_u<R, 2, 0>(d, arena, b0, b1, r, c, red); break;
    case 7: exec_wide_u<R, 2, 1>(d, arena, b0, b1, r, c, red); break;
    case 8: exec_wide_u<R, 2, 2>(d, arena, b0, b1, r, c, red); break;
    case 9: exec_wide_u<R, 3, 0>(d, arena, b0, b1, r, c, red); break;
    case 10: exec_wide_u<R, 3, 1>(d, arena, b0, b1, r, c, red); break;
    case 11: exec_wide_u<R, 3, 2>(d, arena, b0, b1, r, c, red); break;
    case 12: exec_wide_u<R, 4, 0>(d, arena, b0, b1, r, c, red); break;
    case 13: exec_wide_u<R, 4, 1>(d, arena, b0, b1, r, c, red); break;
    case 14: exec_wide_u<R, 4, 2>(d, arena, b0, b1, r, c, red); break;
    default: break;
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

// Executor of OP_ADJOINT ops flagged F_OUTER: every input adjoint of a wide
// bucket whose inputs each lack a different part of the union (an outer
// product of its inputs), in one pass that reads the output adjoint and each
// input once, with every sum in registers.  Union bits: nl lanes (the lowest
// union bits), KI slot bits (unrolled: 2^KI union elements per loop step,
// their loads in flight together), nk loop bits walked per thread in Gray
// order, then block bits.  Every output keeps 2^KI register slots of pairs.
// An output holding the loop bits is flushed after every loop step; the others
// sum over the loop and over block steps that flip only bits they lack, and
// are flushed once.  A flush adds the slots whose bits the output lacks, then
// combines the lanes it lacks (shuffles within the wavefront) and stores each
// remaining value, or adds it with atomics into zeroed memory when the output
// lacks a block bit.  Block ranges as in exec_wide.
template <typename R, int NIN, int KI>
__device__ __forceinline__ void exec_outer(const OpDesc& d, typename CT<R>::E* __restrict__ arena, int64_t blk_begin,
                                           int64_t blk_end, int64_t wg_rank, int64_t wg_count) {
  using E = typename CT<R>::E;
  constexpr int NS = 1 << KI;
  const int tid = threadIdx.x;
  const int nl = d.nl, nk = d.nk;
  const int sbits = 31 - __clz(blockDim.x >> nl);
  const int sub = tid >> nl;
  const int lane = tid & ((1 << nl) - 1);
  const int zk0 = nl + KI, zb0 = nl + KI + nk;
  uint32_t blockbits = 0;
  for (int z = zb0; z < d.nbits - 1; ++z) blockbits |= 1u << d.zbit[z];
  uint32_t mask[NIN], loff[NIN], lsum[NIN], slack[NIN], sst[NIN][KI > 0 ? KI : 1];
  bool hold[NIN], atom[NIN];
  const E* inp[NIN];
  E* outp[NIN];
  uint32_t aheld = 0;  // bits held by an output that sums over the loop
#pragma unroll
  for (int i = 0; i < NIN; ++i) {
    mask[i] = d.in_mask[i];
    inp[i] = arena + d.in_off[i];
    outp[i] = arena + (i ? d.adj_off[i] : 0);
    hold[i] = i > 0 && nk > 0 && ((mask[i] >> d.zbit[zk0]) & 1u);
    atom[i] = (blockbits & ~mask[i]) != 0;
    if (i > 0 && !hold[i]) aheld |= mask[i];
    uint32_t o = 0, ls = 0, sl = 0;
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
#pragma unroll
    for (int j = 0; j < KI; ++j) {
      const uint32_t u = d.zbit[nl + j];
      const bool h = (mask[i] >> u) & 1u;
      sst[i][j] = h ? bit_stride(mask[i], u) : 0u;
      if (!h) sl |= 1u << j;
    }
    loff[i] = o;
    lsum[i] = ls;
    slack[i] = sl;
  }
  // offset of slot s of input i
  auto soff = [&](int i, int s) {
    uint32_t o = 0;
#pragma unroll
    for (int j = 0; j < KI; ++j)
      if ((s >> j) & 1) o += sst[i][j];
    return o;
  };
  const int nloop = 1 << nk;
  const uint32_t base_blk = (uint32_t)blk_begin;
  const int lg_nblk = 31 - __clz((uint32_t)(blk_end - blk_begin));
  const int lg_st = lg_nblk - sbits;
  const int lg_wg = 31 - __clz((uint32_t)wg_count);
  const int lg_chunk = lg_st > lg_wg ? lg_st - lg_wg : 0;
  const int chunk = 1 << lg_chunk;
  const int nchunks = 1 << (lg_st - lg_chunk);
  E acc0[NIN][NS], acc1[NIN][NS];
#pragma unroll
  for (int i = 0; i < NIN; ++i)
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      acc0[i][s] = E{0, 0};
      acc1[i][s] = E{0, 0};
    }
  // add the slots output i lacks, combine its lacked lanes, store or add
  auto flush = [&](int i, uint32_t base) {
#pragma unroll
    for (int j = 0; j < KI; ++j)
      if ((slack[i] >> j) & 1u) {
#pragma unroll
        for (int s = 0; s < NS; ++s)
          if (!((s >> j) & 1)) {
            acc0[i][s] = cadd(acc0[i][s], acc0[i][s | (1 << j)]);
            acc1[i][s] = cadd(acc1[i][s], acc1[i][s | (1 << j)]);
          }
      }
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      if ((uint32_t)s & slack[i]) continue;  // uniform
      E s0 = acc0[i][s], s1 = acc1[i][s];
      for (int j = 0; j < 6; ++j)
        if ((lsum[i] >> j) & 1u) {
          s0 = cadd(s0, shfl_xor_c(s0, 1 << j));
          s1 = cadd(s1, shfl_xor_c(s1, 1 << j));
        }
      if ((lane & lsum[i]) == 0) {
        E* p = outp[i] + base + soff(i, s);
        if (atom[i]) {
          atomic_add_c(p, s0);
          atomic_add_c(p + 1, s1);
        } else {
          store_pair(p, s0, s1);
        }
      }
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      acc0[i][s] = E{0, 0};
      acc1[i][s] = E{0, 0};
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
        E ob[NS], a0[NS][NIN], a1[NS][NIN];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          ob[s] = inp[0][koff[0] + soff(0, s)];
#pragma unroll
          for (int i = 1; i < NIN; ++i) load_pair(inp[i] + koff[i] + soff(i, s), a0[s][i], a1[s][i]);
        }
#pragma unroll
        for (int s = 0; s < NS; ++s) {
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
                acc1[i][s] = cadd(acc1[i][s], e);
              else
                acc0[i][s] = cadd(acc0[i][s], e);
            }
          }
        }
#pragma unroll
        for (int i = 1; i < NIN; ++i)
          if (hold[i]) flush(i, koff[i]);
      }
      if (nxt && !(aheld & nxt)) continue;  // uniform: every summing output carries
#pragma unroll
      for (int i = 1; i < NIN; ++i) {
        if (hold[i] || (nxt && !(mask[i] & nxt))) continue;
        flush(i, boff[i]);
      }
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
  if (d.flags & F_OUTER) {  // planned for complex64 only
    if constexpr (sizeof(R) == 4) {
      if (d.n_in == 3)
        exec_outer<R, 3, 1>(d, arena, b0, b1, r, c);
      else if (d.n_in == 4)
        exec_outer<R, 4, 1>(d, arena, b0, b1, r, c);
    }
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

template <typename R, int MAXNIN>
__device__ __forceinline__ void exec_contract_any(const OpDesc& d, typename CT<R>::E* arena, int64_t b0, int64_t b1,
                                                  int64_t r, int64_t c, RedBuf<typename CT<R>::E>* red) {
  switch (d.n_in) {
    case 1: exec_contract<R, 1>(d, arena, b0, b1, r, c, red); break;
    case 2: exec_contract<R, 2>(d, arena, b0, b1, r, c, red); break;
    case 3: exec_contract<R, 3>(d, arena, b0, b1, r, c, red); break;
    case 4: if constexpr (MAXNIN >= 4) exec_contract<R, 4>(d, arena, b0, b1, r, c, red); break;
    case 5: if constexpr (MAXNIN >= 5) exec_contract<R, 5>(d, arena, b0, b1, r, c, red); break;
    case 6: if constexpr (MAXNIN >= 6) exec_contract<R, 6>(d, arena, b0, b1, r, c, red); break;
    case 7: if constexpr (MAXNIN >= 7) exec_contract<R, 7>(d, arena, b0, b1, r, c, red); break;
    default: if constexpr (MAXNIN >= 8) exec_contract<R, 8>(d, arena, b0, b1, r, c, red); break;
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
__device__ __forceinline__ void exec_result(const OpDesc& d, typename CT<R>::E* arena, const Env& env) {
  using E = typename CT<R>::E;
  double* res = env.res + (int64_t)d.cone * env.res_stride;
  const int ns = d.n_in;
  auto at = [&](int i) -> E* { return arena + d.in_off[i]; };
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
// lds: LDS space for the tile sums of LDS-tiled adjoints.
template <typename R, int MAXNIN, bool WIDE = false>
__device__ __forceinline__ void exec_op(const OpDesc& d, const Env& env, int64_t b0, int64_t b1, int64_t wg_rank,
                                        int64_t wg_count, RedBuf<typename CT<R>::E>* red,
                                        typename CT<R>::E* lds = nullptr) {
  using E = typename CT<R>::E;
  E* arena = reinterpret_cast<E*>(env.arena);
  switch (d.kind) {
    case OP_CONTRACT:
      if constexpr (WIDE) {
        if (d.flags & F_WIDE) {
          exec_wide_any<R>(d, arena, b0, b1, wg_rank, wg_count, red);
          break;
        }
      }
      if constexpr (MAXNIN < 0)
        exec_contract<R, -MAXNIN>(d, arena, b0, b1, wg_rank, wg_count, red);
      else
        exec_contract_any<R, MAXNIN>(d, arena, b0, b1, wg_rank, wg_count, red);
      break;
    case OP_ADJOINT:
      if constexpr (WIDE) exec_adjoint_any<R>(d, arena, b0, b1, wg_rank, wg_count, lds);
      break;
    case OP_LEAF: exec_leaf<R>(d, arena, env, wg_rank, wg_count); break;
    case OP_RESULT:
      if (wg_rank == 0) exec_result<R>(d, arena, env);
      break;
    case OP_ZERO: exec_zero<R>(d, arena, wg_rank, wg_count); break;
    case OP_LEAFGRAD:
      if (wg_rank == 0) exec_leafgrad<R>(d, arena, env);
      break;
    default: break;
  }
}

// ------------------------------------------------------------------ LDS-resident programs
// A light cone whose whole program fits the LDS window runs in one workgroup
// from compact SmallOps.  The ops are read through the scalar cache (uniform
// address, constant address space), so every descriptor field is a scalar
// register and the per-op setup costs a few instructions.
#define QTN_CONST __attribute__((address_space(4)))

// A record loaded through the scalar cache: word by word from the constant
// address space (the address must be uniform across the wavefront).
template <typename T>
__device__ __forceinline__ T load_const(const T* p) {
  static_assert(sizeof(T) % 4 == 0, "records are loaded in 32-bit words");
  const QTN_CONST uint32_t* q = (const QTN_CONST uint32_t*)p;
  T v;
  uint32_t* w = reinterpret_cast<uint32_t*>(&v);
#pragma unroll
  for (int i = 0; i < (int)(sizeof(T) / 4); ++i) w[i] = q[i];
  return v;
}

__device__ __forceinline__ uint32_t nib(uint64_t v, int j) { return (uint32_t)(v >> (4 * j)) & 0xfu; }

// Contraction on one wavefront.  Virtual lane v covers the first nv = n_out +
// ls dimensions (the output element and, when the output has fewer than 64
// elements, the lowest summed dimensions, which are then reduced across the
// wavefront); lane bits are the first min(nv, 6) dimensions, the rest of v is
// a per-lane loop (in Gray-code order).  Each lane walks the summed dimensions
// nv.. in Gray-code order, two at a time (both values of the first), so its
// loads are independent.  Offsets move by XOR: every dimension an input holds
// is one bit of its element index.  An op shared by nparts wavefronts: this
// one takes part `part` of the outer loop (contiguous chunks).
template <typename R, int NIN>
__device__ __forceinline__ void small_contract(const SmallOp& d, typename CT<R>::E* __restrict__ lds,
                                               typename CT<R>::E* __restrict__ arena, int lane, int part = 0,
                                               int nparts = 1) {
  using E = typename CT<R>::E;
  const int nb = d.nbits, no = d.n_out, ns = nb - no;
  const int ls = min(ns, max(0, 6 - no));
  const int nv = no + ls, nk = ns - ls;
  const int nl = min(nv, 6);
  const E* in[NIN];
  uint32_t st0[NIN], off[NIN];
#pragma unroll
  for (int i = 0; i < NIN; ++i) {
    in[i] = lds + d.in_off[i];
    const uint32_t s = nk > 0 ? nib(d.shift[i], nv) : 0xfu;
    st0[i] = s == 0xfu ? 0u : (1u << s);
    uint32_t o = 0;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      const uint32_t sj = nib(d.shift[i], j);
      if (j < nl && sj != 0xfu) o |= ((uint32_t)(lane >> j) & 1u) << sj;
    }
    off[i] = o;
  }
  const bool active = lane < (1 << nl);
  const int nouter = 1 << (nv - nl);
  const int chunk = (nouter + nparts - 1) / nparts;
  const int h0 = min(nouter, part * chunk), h1 = min(nouter, h0 + chunk);
  uint32_t g = (uint32_t)(h0 ^ (h0 >> 1));  // Gray code of the outer loop (dimensions 6 .. nv - 1)
  for (int t = 0; t < nv - nl; ++t)
    if ((g >> t) & 1u) {
#pragma unroll
      for (int i = 0; i < NIN; ++i) {
        const uint32_t s = nib(d.shift[i], 6 + t);
        off[i] ^= s == 0xfu ? 0u : (1u << s);
      }
    }
  for (int h = h0; h < h1; ++h) {
    if (h > h0) {
      const int t = __ffs(h) - 1;
      g ^= 1u << t;
#pragma unroll
      for (int i = 0; i < NIN; ++i) {
        const uint32_t s = nib(d.shift[i], 6 + t);
        off[i] ^= s == 0xfu ? 0u : (1u << s);
      }
    }
    E acc0 = {0, 0}, acc1 = {0, 0};
    if (active) {
      uint32_t o2[NIN];
#pragma unroll
      for (int i = 0; i < NIN; ++i) o2[i] = off[i];
      if (nk == 0) {
        E p = in[0][o2[0]];
#pragma unroll
        for (int i = 1; i < NIN; ++i) p = cmul(p, in[i][o2[i]]);
        acc0 = p;
      } else {
        const int nit = 1 << (nk - 1);
        for (int it = 0; it < nit; ++it) {
          if (it) {
            const int j = nv + __ffs(it);  // Gray code over dimensions nv + 1 ..
#pragma unroll
            for (int i = 0; i < NIN; ++i) {
              const uint32_t s = nib(d.shift[i], j);
              o2[i] ^= s == 0xfu ? 0u : (1u << s);
            }
          }
          E a[NIN], b[NIN];
#pragma unroll
          for (int i = 0; i < NIN; ++i) {
            a[i] = in[i][o2[i]];
            b[i] = in[i][o2[i] ^ st0[i]];
          }
          E p = a[0], q = b[0];
#pragma unroll
          for (int i = 1; i < NIN; ++i) {
            p = cmul(p, a[i]);
            q = cmul(q, b[i]);
          }
          acc0 = cadd(acc0, p);
          acc1 = cadd(acc1, q);
        }
      }
    }
    acc0 = cadd(acc0, acc1);
    // summed lane dimensions no .. nv - 1 (then nv <= 6), lowest first: each
    // step adds the value of lane + 2^j, so the lanes with all of these bits
    // zero (the ones that store) end with the whole sum
    if (no <= 0 && nv > 0) acc0 = cadd(acc0, lane_down_c<0>(acc0));
    if (no <= 1 && nv > 1) acc0 = cadd(acc0, lane_down_c<1>(acc0));
    if (no <= 2 && nv > 2) acc0 = cadd(acc0, lane_down_c<2>(acc0));
    if (no <= 3 && nv > 3) acc0 = cadd(acc0, lane_down_c<3>(acc0));
    if (no <= 4 && nv > 4) acc0 = cadd(acc0, lane_down_c<4>(acc0));
    if (no <= 5 && nv > 5) acc0 = cadd(acc0, lane_down_c<5>(acc0));
    const uint32_t v = (uint32_t)lane | (g << 6);
    if (active && ((v >> no) & ((1u << ls) - 1u)) == 0) {
      const uint32_t o = v & ((1u << no) - 1u);
      if (d.flags & SF_GOUT)
        arena[d.gout + o] = acc0;  // a leaf-table adjoint, for the leaf-gradient launch
      else
        lds[d.out_off + o] = acc0;
    }
  }
}

template <typename R>
__device__ __forceinline__ void small_contract_any(const SmallOp& d, typename CT<R>::E* lds,
                                                   typename CT<R>::E* arena, int lane, int part, int nparts) {
  switch (d.n_in) {
    case 1: small_contract<R, 1>(d, lds, arena, lane, part, nparts); break;
    case 2: small_contract<R, 2>(d, lds, arena, lane, part, nparts); break;
    case 3: small_contract<R, 3>(d, lds, arena, lane, part, nparts); break;
    case 4: small_contract<R, 4>(d, lds, arena, lane, part, nparts); break;
    case 5: small_contract<R, 5>(d, lds, arena, lane, part, nparts); break;
    case 6: small_contract<R, 6>(d, lds, arena, lane, part, nparts); break;
    case 7: small_contract<R, 7>(d, lds, arena, lane, part, nparts); break;
    default: small_contract<R, 8>(d, lds, arena, lane, part, nparts); break;
  }
}

// A table's leaf references (L <= LM <= 64) into uniform registers: lane q
// loads reference q (one load for all of them), readlane hands each to the
// wavefront; references beyond L read as zero.
template <int LM>
__device__ __forceinline__ void load_refs(const LeafRef* refs, int L, int lane, LeafRef (&lr)[LM]) {
  const uint32_t mine = lane < L ? reinterpret_cast<const uint32_t*>(refs)[lane] : 0u;
#pragma unroll
  for (int q = 0; q < LM; ++q) {
    const uint32_t r = (uint32_t)__builtin_amdgcn_readlane((int)mine, q);
    lr[q].kind = (int16_t)(r & 0xffffu);
    lr[q].pa = (int8_t)((r >> 16) & 0xffu);
    lr[q].pb = (int8_t)(r >> 24);
  }
}
static_assert(sizeof(LeafRef) == 4, "a leaf reference is one 32-bit word");

// Leaf-product table on one wavefront (lane 0..63): entry e of out = product
// over the table's L leaves of leaf[e restricted to the leaf's two indices].
// LM >= L: the body is branch-free (missing leaves multiply by one), so every
// value load of an entry is in flight at once; references read once.
template <typename R, int LM>
__device__ __forceinline__ void leaf_table_wave_m(typename CT<R>::E* out, int n, const LeafRef* refs, int L,
                                                  const typename CT<R>::E* vals, int lane) {
  using E = typename CT<R>::E;
  LeafRef lr[LM];
  load_refs<LM>(refs, L, lane, lr);
  for (int e = lane; e < n; e += 64) {
    E v[LM];
#pragma unroll
    for (int q = 0; q < LM; ++q) {
      const int hi = lr[q].pb >= 0 ? ((e >> (lr[q].pb & 31)) & 1) << 1 : 0;
      v[q] = vals[lr[q].kind * 4 + (((e >> lr[q].pa) & 1) | hi)];
    }
    E p = {1, 0};
#pragma unroll
    for (int q = 0; q < LM; ++q)
      if (q < L) p = cmul(p, v[q]);
    out[e] = p;
  }
}

template <typename R>
__device__ __forceinline__ void leaf_table_wave(typename CT<R>::E* out, int n, const LeafRef* refs, int L,
                                                const typename CT<R>::E* vals, int lane) {
  using E = typename CT<R>::E;
  if (L <= 4) {
    leaf_table_wave_m<R, 4>(out, n, refs, L, vals, lane);
  } else if (L <= 8) {
    leaf_table_wave_m<R, 8>(out, n, refs, L, vals, lane);
  } else if (L <= 16) {
    leaf_table_wave_m<R, 16>(out, n, refs, L, vals, lane);
  } else {
    for (int e = lane; e < n; e += 64) {
      E p = {1, 0};
      for (int r = 0; r < L; ++r) {
        const LeafRef Lr = refs[r];
        int idx = (e >> Lr.pa) & 1;
        if (Lr.pb >= 0) idx |= ((e >> Lr.pb) & 1) << 1;
        p = cmul(p, vals[Lr.kind * 4 + idx]);
      }
      out[e] = p;
    }
  }
}

// dR/dtheta += sum_e Lbar[e] * (derivative of one leaf) * (the other leaves),
// by one wavefront (lane 0..63) over the n entries of one leaf-product table
// with L <= LM leaves.  Per entry: every leaf value and derivative loaded at
// once, suffix products of the leaves, then one pass with the running prefix
// (3L complex multiplies instead of L^2), branch-free; leaves come sorted by
// kind, so one wavefront sum and one atomic per angle.
template <typename R, int LM>
__device__ __forceinline__ void leafgrad_wave_m(const typename CT<R>::E* lbar, int n, const LeafRef* refs, int L,
                                                const typename CT<R>::E* vals, const typename CT<R>::E* dvals,
                                                double* res, int p, int lane) {
  using E = typename CT<R>::E;
  LeafRef lr[LM];
  load_refs<LM>(refs, L, lane, lr);
  int slot[LM];
#pragma unroll
  for (int q = 0; q < LM; ++q) slot[q] = q < L ? theta_slot(lr[q].kind, p) : -1;
  double sxd[LM], syd[LM];
#pragma unroll
  for (int q = 0; q < LM; ++q) sxd[q] = syd[q] = 0.0;
  for (int e = lane; e < n; e += 64) {
    E v[LM], dv[LM];
#pragma unroll
    for (int q = 0; q < LM; ++q) {
      const int hi = lr[q].pb >= 0 ? ((e >> (lr[q].pb & 31)) & 1) << 1 : 0;
      const int k = lr[q].kind * 4 + (((e >> lr[q].pa) & 1) | hi);
      v[q] = q < L ? vals[k] : E{1, 0};
      dv[q] = dvals[k];
    }
    E suf[LM + 1];
    suf[LM] = E{1, 0};
#pragma unroll
    for (int q = LM - 1; q >= 0; --q) suf[q] = cmul(v[q], suf[q + 1]);
    E pre = lbar[e];
#pragma unroll
    for (int q = 0; q < LM; ++q) {
      const E t = cmul(cmul(pre, dv[q]), suf[q + 1]);
      sxd[q] += (double)t.x;
      syd[q] += (double)t.y;
      pre = cmul(pre, v[q]);
    }
  }
  int cur = -1;
  double sx = 0, sy = 0;
#pragma unroll
  for (int q = 0; q <= LM; ++q) {
    const int sl = q < LM ? slot[q] : -2;  // uniform across the wavefront
    if (sl == -1) continue;
    if (sl != cur && cur >= 0) {
      const double wx = wave_sum(sx), wy = wave_sum(sy);
      if (lane == 0) {
        atomicAdd(res + cur, wx);
        atomicAdd(res + cur + 1, wy);
      }
    }
    if (sl == -2) break;
    if (sl != cur) {
      cur = sl;
      sx = sy = 0;
    }
    sx += sxd[q];
    sy += syd[q];
  }
}

// (LMAX: the caller's bound on L; a smaller bound leaves the larger variants
// out of the kernel, and with them their register footprint)
template <typename R, int LMAX = 64>
__device__ __forceinline__ void leafgrad_wave(const typename CT<R>::E* lbar, int n, const LeafRef* refs, int L,
                                              const typename CT<R>::E* vals, const typename CT<R>::E* dvals,
                                              double* res, int p, int lane) {
  using E = typename CT<R>::E;
  if (L <= 4) {
    leafgrad_wave_m<R, 4>(lbar, n, refs, L, vals, dvals, res, p, lane);
  } else if (LMAX <= 8 || L <= 8) {
    leafgrad_wave_m<R, 8>(lbar, n, refs, L, vals, dvals, res, p, lane);
  } else if (L <= 16) {
    leafgrad_wave_m<R, 16>(lbar, n, refs, L, vals, dvals, res, p, lane);
  } else {
    // many leaves (rare): one pass over the entries per leaf with an angle
    for (int r = 0; r < L; ++r) {
      const int slot = theta_slot(refs[r].kind, p);
      if (slot < 0) continue;  // uniform across the wavefront
      double ax = 0, ay = 0;
      for (int e = lane; e < n; e += 64) {
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

// Cone value R = product of the scalars; with SF_GRAD also the seed of each
// scalar (product of the others) and zeroed gradient accumulators.  One
// wavefront.
template <typename R>
__device__ __forceinline__ void small_result(const SmallOp& d, typename CT<R>::E* lds, const Env& env, int lane) {
  using E = typename CT<R>::E;
  double* res = env.res + (int64_t)d.cone * env.res_stride;
  const int ns = d.n_in;  // <= 4 scalars (one per connected component)
  double2 x[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const E v = s < ns ? lds[d.in_off[s]] : E{1, 0};
    x[s] = make_double2(v.x, v.y);
  }
  if (lane == 0) {
    const double2 prod = cmul(cmul(x[0], x[1]), cmul(x[2], x[3]));
    res[0] = prod.x;
    res[1] = prod.y;
  }
  if (d.flags & SF_GRAD) {
    // seed of scalar s: product of the other scalars (lane s)
#pragma unroll
    for (int s = 0; s < 4; ++s)
      if (s < ns && lane == s) {
        double2 seed = make_double2(1, 0);
#pragma unroll
        for (int t = 0; t < 4; ++t)
          if (t != s) seed = cmul(seed, x[t]);
        E o;
        o.x = (R)seed.x;
        o.y = (R)seed.y;
        lds[d.in_off[4 + s]] = o;
      }
    for (int i = lane; i < 4 * env.p; i += 64) res[2 + i] = 0.0;
  }
}

// One cone's LDS-resident program small[lo, hi) on the whole workgroup.  Each
// wavefront reads the ops itself, one op (32 words) per load, lane q holding
// word q: the next op's load is issued before the current op runs, so it
// arrives during it, and no wavefront waits for another to fetch the
// program.  Fields go to scalar registers by readlane, only those the op's
// kind needs (a contraction: the header, its inputs' dimension maps, the
// global output offset when it has one).  The leaf-block copy runs on all
// threads; every other op on its wavefront (ops between two barriers are
// independent, so the wavefronts run them side by side).  The workgroup has a
// power-of-two number of wavefronts (1, 2, 4 or 8).
template <typename R>
__device__ __forceinline__ void run_small(const SmallOp* small, int lo, int hi, typename CT<R>::E* lds,
                                          const Env& env) {
  using E = typename CT<R>::E;
  constexpr int NW = (int)(sizeof(SmallOp) / 4);  // 32 words per op
  static_assert(NW == 32, "an op is read by half a wavefront");
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nw = blockDim.x >> 6;
  const uint32_t* words = reinterpret_cast<const uint32_t*>(small);
  uint32_t cur = words[(size_t)lo * NW + (lane & (NW - 1))];
  for (int k = lo; k < hi; ++k) {
    const uint32_t nxt = k + 1 < hi ? words[(size_t)(k + 1) * NW + (lane & (NW - 1))] : 0u;
    auto W = [&](int q) { return (uint32_t)__builtin_amdgcn_readlane((int)cur, q); };
    // kind, flags and wavefront first: the other wavefronts skip the op here
    const uint32_t w0 = W(0), w1 = W(1);
    const uint32_t kind = w0 & 0xffu, flags = w1 & 0xffu, owner = (w1 >> 8) & 0xffu;
    if (k > lo && (flags & SF_SYNC)) __syncthreads();
    const bool split = flags & SF_SPLIT;
    if (kind != S_COPYIN && !split && (int)(owner & (uint32_t)(nw - 1)) != wave) {
      cur = nxt;
      continue;
    }
    SmallOp d;
    uint32_t* dw = reinterpret_cast<uint32_t*>(&d);
    dw[0] = w0;
    dw[1] = w1;
#pragma unroll
    for (int q = 2; q < 8; ++q) dw[q] = W(q);
    if (kind == S_CONTRACT) {
      const int nin = (int)((w0 >> 8) & 0xffu);
#pragma unroll
      for (int q = 0; q < 16; ++q)
        if (q < 2 * nin) dw[8 + q] = W(8 + q);
      if (flags & SF_GOUT) {
        dw[24] = W(24);
        dw[25] = W(25);
      }
      small_contract_any<R>(d, lds, reinterpret_cast<E*>(env.arena), lane, split ? wave : 0, split ? nw : 1);
    } else {
#pragma unroll
      for (int q = 8; q < NW; ++q) dw[q] = W(q);
      if (kind == S_COPYIN) {
        const E* src = reinterpret_cast<const E*>(env.arena) + d.gout;
        for (int t = threadIdx.x; t < d.aux1; t += blockDim.x) lds[t] = src[t];
      } else if (kind == S_RESULT) {
        small_result<R>(d, lds, env, lane);
      }
    }
    cur = nxt;
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

}  // namespace qtn
