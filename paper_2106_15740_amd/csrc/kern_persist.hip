// Persistent work-queue kernel of the batched sweep for one element type and
// one executor set: built with QTN_REAL = float / double and QTN_WIDE = 0 / 1.
#include "exec.hpp"

namespace qtn {

constexpr int DESC_CHUNK = 16;

// Persistent sweep: workgroups pop items from a device queue in topological
// order; an item waits until its node counter is zero, runs, then releases
// its successor nodes.  Every item waits only on items earlier in the queue,
// which were already taken by running workgroups, so the sweep always drains.
// WIDE: the plan has F_WIDE ops (a separate instantiation keeps the register
// budget of narrow-only sweeps unchanged).
template <typename R, int MAXNIN, bool WIDE>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 4 : 1, 8)))
persistent_kernel(const OpDesc* __restrict__ ops, const QItem* __restrict__ items, int n_items,
                  const int32_t* __restrict__ succ, int32_t* ctl, Env env, long long spin_limit) {
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
            exec_op<R, MAXNIN, WIDE>(d, env, b0, b1, 0, 1, &red, reinterpret_cast<E*>(dyn_lds));
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
hipError_t launch_persistent_t(int max_nin, const OpDesc* ops, const QItem* items, int n_items, const int32_t* succ,
                               int32_t* ctl, const Env& env, int threads, int grid, size_t lds_bytes,
                               long long spin_limit, hipStream_t st) {
  if (max_nin <= 3)
    return launch_persistent_m<R, 3, W>(ops, items, n_items, succ, ctl, env, threads, grid, lds_bytes, spin_limit, st);
  if (max_nin <= 5)
    return launch_persistent_m<R, 5, W>(ops, items, n_items, succ, ctl, env, threads, grid, lds_bytes, spin_limit, st);
  return launch_persistent_m<R, 8, W>(ops, items, n_items, succ, ctl, env, threads, grid, lds_bytes, spin_limit, st);
}

template hipError_t launch_persistent_t<QTN_REAL, QTN_WIDE>(int, const OpDesc*, const QItem*, int, const int32_t*,
                                                            int32_t*, const Env&, int, int, size_t, long long,
                                                            hipStream_t);

}  // namespace qtn
