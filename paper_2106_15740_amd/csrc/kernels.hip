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
#include <mutex>

#include "exec.hpp"

namespace qtn {

// Leaf-product tables (OP_LEAF, GRAD false) or leaf gradients (OP_LEAFGRAD,
// GRAD true, tables of at most LMAX leaves) of every cone, one wavefront per
// op: the tables have a few to a few hundred entries, so a whole workgroup per
// op would idle.  Separate kernels, so the tables and the gradients of tables
// with few leaves keep the small register footprint (and the occupancy) of
// their simpler bodies.
template <typename R, bool GRAD, int LMAX>
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
  __shared__ E s_vals[NV], s_dvals[GRAD ? NV : 1];
  const int nv = 4 * (3 + 4 * env.p);
  for (int i = threadIdx.x; i < nv && i < NV; i += blockDim.x) {
    s_vals[i] = reinterpret_cast<const E*>(env.leafvals)[i];
    if (GRAD) s_dvals[i] = reinterpret_cast<const E*>(env.dleafvals)[i];
  }
  __syncthreads();
  E* arena = reinterpret_cast<E*>(env.arena);
  for (int op = lo + wave; op < hi; op += nwaves) {
    const OpDesc& d = ops[op];
    const int64_t n = int64_t(1) << d.nbits;
    const LeafRef* refs = env.leafrefs + d.aux0;
    if (!GRAD)
      leaf_table_wave<R>(arena + d.out_off, (int)n, refs, d.aux1, s_vals, lane);
    else
      leafgrad_wave<R, LMAX>(arena + d.in_off[0], (int)n, refs, d.aux1, s_vals, s_dvals,
                       env.res + (int64_t)d.cone * env.res_stride, env.p, lane);
  }
}

// LDS-resident light cones: workgroup k runs the whole program
// small[items[2k], items[2k + 1]) of one cone with every tensor in its LDS
// window (items are ordered longest first).
template <typename R>
__global__ void __launch_bounds__(512) small_kernel(const SmallOp* __restrict__ small, const int32_t* __restrict__ items,
                                                    Env env) {
  using E = typename CT<R>::E;
  extern __shared__ __align__(16) char dyn_lds[];
  const int2 r = load_const(reinterpret_cast<const int2*>(items) + blockIdx.x);
  run_small<R>(small, r.x, r.y, reinterpret_cast<E*>(dyn_lds), env);
}

// Copy of a few hundred bytes between device memory and mapped pinned host
// memory (leaf values in, results out): a kernel node keeps the sweep's
// graph free of copy-engine transfers and their start-up latency.
__global__ void __launch_bounds__(256) small_copy_kernel(const uint32_t* __restrict__ src, uint32_t* __restrict__ dst,
                                                         int n, int32_t* ctl, const int32_t* __restrict__ ctl_init,
                                                         int n_nodes) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = src[i];
  if (ctl)
    for (int i = threadIdx.x; i < n_nodes + 2; i += blockDim.x) ctl[i] = i < 2 ? 0 : ctl_init[i - 2];
}

// Plain device copy (16-byte words, grid-stride): the achievable-bandwidth
// reference the contraction kernels are compared against.  Each thread keeps
// U 16-byte loads in flight (issued before the first store); consecutive
// threads touch consecutive words, so every load and store is coalesced.
template <int U>
__global__ void __launch_bounds__(256) copy_kernel(const uint4* __restrict__ src, uint4* __restrict__ dst, size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  for (; i + (U - 1) * stride < n; i += U * stride) {
    uint4 v[U];
#pragma unroll
    for (int k = 0; k < U; ++k) v[k] = src[i + k * stride];
#pragma unroll
    for (int k = 0; k < U; ++k) dst[i + k * stride] = v[k];
  }
  for (; i < n; i += stride) dst[i] = src[i];
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
  // all 1 + 2p sums in one pass over the cones (p <= 16), then one
  // wavefront reduction each and a sum over the wavefronts
  constexpr int MAXV = 1 + 2 * 16;
  constexpr int MAXW = 1024 / 64;
  __shared__ double part[MAXV][MAXW];
  const int nv = 1 + (with_grad ? 2 * p : 0);
  double acc[MAXV];
#pragma unroll
  for (int v = 0; v < MAXV; ++v) acc[v] = 0.0;
  for (int c = threadIdx.x; c < n_cones; c += blockDim.x) {
    const double* r = res + (int64_t)c * res_stride;
    if (zz_out) {
      E z;
      z.x = (R)r[0];
      z.y = (R)r[1];
      zz_out[c] = z;
    }
    acc[0] += 0.5 * (1.0 - r[0]);
#pragma unroll
    for (int v = 1; v < MAXV; ++v)
      if (v < nv) acc[v] -= 0.5 * r[2 + 2 * (v - 1)];
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
#pragma unroll
  for (int v = 0; v < MAXV; ++v)
    if (v < nv) {
      const double t = wave_sum(acc[v]);
      if (lane == 0) part[v][wave] = t;
    }
  __syncthreads();
  if (threadIdx.x < nv) {
    double t = 0;
    for (int w = 0; w < nw; ++w) t += part[threadIdx.x][w];
    fin[threadIdx.x] = t;
    if (host_fin) host_fin[threadIdx.x] = t;
  }
  // the queue head and the persistent kernel's error flag, next to the results
  if (host_ctl && threadIdx.x < 2) host_ctl[threadIdx.x] = ctl ? ctl[threadIdx.x] : 0;
}

// ------------------------------------------------------------------ static scratch
// Device workspace of the allocation-free entry point: one array per GPU,
// held until the process ends.  Host code must never pass `scratch` itself to
// a kernel (in host code the name is a host-side stand-in, not a device
// address): scratch_address() looks up the device address once per device
// with that device current and every later use goes through it.
static __device__ __align__(256) char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t scratch_address(int device, void** ptr) {
  *ptr = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = p;
  }
  *ptr = g_scratch_ptr[device];
  return hipSuccess;
}

// ------------------------------------------------------------------ host launchers
hipError_t launch_op(bool c128, const OpDesc* d_ops, const OpDesc& h, int op, const Env& env, int threads,
                     int max_grid, hipStream_t st) {
  return c128 ? launch_op_t<double>(d_ops, h, op, env, threads, max_grid, st)
              : launch_op_t<float>(d_ops, h, op, env, threads, max_grid, st);
}

hipError_t launch_batch(bool c128, bool grad, int lmax, const OpDesc* d_ops, int lo, int hi, const Env& env,
                        hipStream_t st, int32_t* ctl, const int32_t* ctl_init, int n_nodes) {
  if (hi <= lo && !ctl) return hipSuccess;
  // 4 wavefronts per workgroup, one op each
  const int grid = std::max(1, std::min(std::max(hi - lo, 0) / 4 + 1, 4096));
#define QTN_LEAF(R, G, LM) \
  hipLaunchKernelGGL((leaf_batch_kernel<R, G, LM>), dim3(grid), dim3(256), 0, st, d_ops, lo, hi, env, ctl, ctl_init, \
                     n_nodes)
  if (c128) {
    if (!grad)
      QTN_LEAF(double, false, 64);
    else if (lmax <= 8)
      QTN_LEAF(double, true, 8);
    else
      QTN_LEAF(double, true, 64);
  } else {
    if (!grad)
      QTN_LEAF(float, false, 64);
    else if (lmax <= 8)
      QTN_LEAF(float, true, 8);
    else
      QTN_LEAF(float, true, 64);
  }
#undef QTN_LEAF
  return hipGetLastError();
}

hipError_t launch_small_copy(const void* src, void* dst, size_t bytes, hipStream_t st, int32_t* ctl,
                             const int32_t* ctl_init, int n_nodes) {
  if (bytes == 0 && !ctl) return hipSuccess;
  if (bytes % 4 || bytes > (size_t(1) << 20)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(small_copy_kernel, dim3(1), dim3(256), 0, st, reinterpret_cast<const uint32_t*>(src),
                     reinterpret_cast<uint32_t*>(dst), (int)(bytes / 4), ctl, ctl_init, n_nodes);
  return hipGetLastError();
}

hipError_t launch_copy(const void* src, void* dst, size_t n16, int grid, int unroll, hipStream_t st) {
  if (n16 == 0) return hipSuccess;
  const dim3 g(std::max(1, grid));
  const uint4* s = reinterpret_cast<const uint4*>(src);
  uint4* d = reinterpret_cast<uint4*>(dst);
  if (unroll >= 4)
    hipLaunchKernelGGL(copy_kernel<4>, g, dim3(256), 0, st, s, d, n16);
  else if (unroll == 2)
    hipLaunchKernelGGL(copy_kernel<2>, g, dim3(256), 0, st, s, d, n16);
  else
    hipLaunchKernelGGL(copy_kernel<1>, g, dim3(256), 0, st, s, d, n16);
  return hipGetLastError();
}

hipError_t launch_reset(int32_t* ctl, const int32_t* init, int n_nodes, hipStream_t st) {
  int grid = (n_nodes + 2 + 255) / 256;
  if (grid > 1024) grid = 1024;
  hipLaunchKernelGGL(reset_ctl_kernel, dim3(grid), dim3(256), 0, st, ctl, init, n_nodes);
  return hipGetLastError();
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

template <typename R>
static hipError_t launch_small_t(const SmallOp* small, const int32_t* items, int n_items, const Env& env, int threads,
                                 size_t lds_bytes, hipStream_t st) {
  if (lds_bytes > 0) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&small_kernel<R>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(small_kernel<R>, dim3(n_items), dim3(threads), lds_bytes, st, small, items, env);
  return hipGetLastError();
}

hipError_t launch_small(bool c128, const SmallOp* small, const int32_t* items, int n_items, const Env& env,
                        int threads, size_t lds_bytes, hipStream_t st) {
  if (n_items <= 0) return hipSuccess;
  return c128 ? launch_small_t<double>(small, items, n_items, env, threads, lds_bytes, st)
              : launch_small_t<float>(small, items, n_items, env, threads, lds_bytes, st);
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
