// One-op-per-launch kernels (the plain per-edge loop and standalone timing)
// for one element type: built once with QTN_REAL=float and once with
// QTN_REAL=double.
#include "exec.hpp"

namespace qtn {

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

// One outer-product OP_ADJOINT op per launch (KI register slot bits).
template <typename R, int NIN, int KI>
__global__ void __launch_bounds__(512) outer_kernel(const OpDesc* __restrict__ ops, int op, Env env) {
  __shared__ OpDesc d;
  stage_desc(d, ops, op);
  const int64_t nblocks = int64_t(1) << d.nb;
  exec_outer<R, NIN, KI>(d, reinterpret_cast<typename CT<R>::E*>(env.arena), 0, nblocks, xcd_rank(), gridDim.x);
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

template <typename R>
hipError_t launch_op_t(const OpDesc* d_ops, const OpDesc& h, int op, const Env& env, int threads, int max_grid,
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
  if (h.kind == OP_ADJOINT && (h.flags & F_OUTER)) {  // planned for complex64 only
    if constexpr (sizeof(R) != 4) return hipErrorInvalidValue;
    if (h.nu != 1) return hipErrorInvalidValue;
    if (h.n_in == 3)
      hipLaunchKernelGGL((outer_kernel<R, 3, 1>), g, b, 0, st, d_ops, op, env);
    else if (h.n_in == 4)
      hipLaunchKernelGGL((outer_kernel<R, 4, 1>), g, b, 0, st, d_ops, op, env);
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
    const int ns = !(h.in_mask[0] & 1u) ? (h.n_in > 1 && !(h.in_mask[1] & 1u) ? 2 : 1) : 0;
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
    switch (h.n_in * 3 + ns) {
      case 3: QTN_WIDE_U(1, 0); break;
      case 4: QTN_WIDE_U(1, 1); break;
      case 6: QTN_WIDE_U(2, 0); break;
      case 7: QTN_WIDE_U(2, 1); break;
      case 8: QTN_WIDE_U(2, 2); break;
      case 9: QTN_WIDE_U(3, 0); break;
      case 10: QTN_WIDE_U(3, 1); break;
      case 11: QTN_WIDE_U(3, 2); break;
      case 12: QTN_WIDE_U(4, 0); break;
      case 13: QTN_WIDE_U(4, 1); break;
      case 14: QTN_WIDE_U(4, 2); break;
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

template hipError_t launch_op_t<QTN_REAL>(const OpDesc*, const OpDesc&, int, const Env&, int, int, hipStream_t);

}  // namespace qtn
