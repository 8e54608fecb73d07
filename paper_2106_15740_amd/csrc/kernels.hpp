// Launch interface of the HIP kernels (host side).
#pragma once

#include <hip/hip_runtime.h>

#include "opdesc.hpp"

namespace qtn {

// Pointers every kernel needs.  All device pointers.
struct Env {
  void* arena;              // tensor elements (complex64 or complex128)
  double* res;              // per cone: R (re, im), dR/dgamma_l, dR/dbeta_l (re, im)
  const void* leafvals;     // [4p+3][4] leaf entries, element type (p <= 16)
  const void* dleafvals;    // [4p+3][4] their derivatives in the leaf's angle
  const LeafRef* leafrefs;
  int p;
  int res_stride;           // 2 + 4p doubles
};

hipError_t launch_op(bool c128, const OpDesc* d_ops, const OpDesc& h, int op, const Env& env, int threads,
                     int max_grid, hipStream_t st);
// ops [lo, hi) (all OP_LEAF, or with grad all OP_LEAFGRAD of tables with at
// most lmax leaves), one wavefront each; with ctl, the same launch resets the
// persistent sweep's queue head, error flag and node counters (n_nodes of
// them, from ctl_init)
hipError_t launch_batch(bool c128, bool grad, int lmax, const OpDesc* d_ops, int lo, int hi, const Env& env,
                        hipStream_t st, int32_t* ctl = nullptr, const int32_t* ctl_init = nullptr, int n_nodes = 0);
// bytes (a multiple of 4, <= 1 MiB) from src to dst with one workgroup;
// either side may be mapped pinned host memory.  With ctl, the same launch
// resets the persistent sweep's queue head, error flag and node counters.
hipError_t launch_small_copy(const void* src, void* dst, size_t bytes, hipStream_t st, int32_t* ctl = nullptr,
                             const int32_t* ctl_init = nullptr, int n_nodes = 0);
// n16 16-byte words from src to dst (non-overlapping), `grid` workgroups of
// 256 threads, `unroll` (1, 2 or 4) loads in flight per thread
hipError_t launch_copy(const void* src, void* dst, size_t n16, int grid, int unroll, hipStream_t st);
hipError_t launch_reset(int32_t* ctl, const int32_t* init, int n_nodes, hipStream_t st);
// wide: some op carries F_WIDE; max_nin: the largest input count of any
// contraction op in the items; lds_bytes: dynamic LDS window of LDS-resident
// items (0: none)
hipError_t launch_persistent(bool c128, bool wide, int max_nin, const OpDesc* ops, const QItem* items, int n_items,
                             const int32_t* succ, int32_t* ctl, const Env& env, int threads, int grid,
                             size_t lds_bytes, long long spin_limit, hipStream_t st);
// LDS-resident light cones: one workgroup per program small[items[2k],
// items[2k + 1]), the LDS window lds_bytes
hipError_t launch_small(bool c128, const SmallOp* small, const int32_t* items, int n_items, const Env& env,
                        int threads, size_t lds_bytes, hipStream_t st);
// Per-element-type launchers, each instantiated in its own translation unit
// (kern_ops.hip, kern_persist.hip) so the kernels compile in parallel.
template <typename R>
hipError_t launch_op_t(const OpDesc* d_ops, const OpDesc& h, int op, const Env& env, int threads, int max_grid,
                       hipStream_t st);
template <typename R, bool W>
hipError_t launch_persistent_t(int max_nin, const OpDesc* ops, const QItem* items, int n_items, const int32_t* succ,
                               int32_t* ctl, const Env& env, int threads, int grid, size_t lds_bytes,
                               long long spin_limit, hipStream_t st);
extern template hipError_t launch_op_t<float>(const OpDesc*, const OpDesc&, int, const Env&, int, int, hipStream_t);
extern template hipError_t launch_op_t<double>(const OpDesc*, const OpDesc&, int, const Env&, int, int, hipStream_t);
extern template hipError_t launch_persistent_t<float, false>(int, const OpDesc*, const QItem*, int, const int32_t*,
                                                             int32_t*, const Env&, int, int, size_t, long long,
                                                             hipStream_t);
extern template hipError_t launch_persistent_t<float, true>(int, const OpDesc*, const QItem*, int, const int32_t*,
                                                            int32_t*, const Env&, int, int, size_t, long long,
                                                            hipStream_t);
extern template hipError_t launch_persistent_t<double, false>(int, const OpDesc*, const QItem*, int, const int32_t*,
                                                              int32_t*, const Env&, int, int, size_t, long long,
                                                              hipStream_t);
extern template hipError_t launch_persistent_t<double, true>(int, const OpDesc*, const QItem*, int, const int32_t*,
                                                             int32_t*, const Env&, int, int, size_t, long long,
                                                             hipStream_t);

// Bytes of the static device scratch used by the allocation-free entry
// point, and its device address on `device` (looked up once per device with
// that device current, then cached).
constexpr size_t kScratchBytes = size_t(64) << 20;
hipError_t scratch_address(int device, void** ptr);

// E, dE/dgamma, dE/dbeta into fin and, when host_fin is given, into mapped
// pinned host memory, with ctl[0..1] (or zeros without ctl) into host_ctl
hipError_t launch_final(bool c128, const double* res, int res_stride, int n_cones, int p, int with_grad, void* zz_out,
                        double* fin, double* host_fin, const int32_t* ctl, int32_t* host_ctl, hipStream_t st);

}  // namespace qtn
