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
