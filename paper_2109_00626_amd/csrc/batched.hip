// Batched interface sweeps: many independent (X, Y) pairs of uneven order,
// mode sizes and ranks in one persistent launch.
//
// Each workgroup owns a list of pairs fixed by the host planner (longest
// first onto the least-loaded workgroup), so there is no device-side queue
// and no atomic.  For a pair of order N the workgroup sweeps right to left:
//   V_N = [1],  V_k = sum_i G_x^(k)[:, i, :] V_{k+1} G_y^(k)[:, i, :]^T  (k >= 1),
// stores V_{N-2} (the junction of the contraction over the last two
// positions) when asked, then forms W_1 = sum_i G_x^(0)[0, i, :]^T G_y^(0)[0, i, :]
// and finishes <X, Y> = sum W_1 .* V_1 in FP64.  Each step is the
// chained-MFMA step of sweep_steps.hpp; the two interface buffers of a pair
// live in LDS when they fit the workgroup's budget, else in the workgroup's
// slice of plan memory.
#include "sweep_steps.hpp"
#include "ttc_batch.h"
#include "ttc_device.hpp"

namespace ttc {

template <typename Tin>
__device__ void load_pair(const BatchArgs& a, int p, TTDev* x, TTDev* y, long* jout) {
  // descriptors are read into registers/LDS-free locals by thread-uniform loads
  const PairDev pd = a.pairs[p];
  x->order = y->order = pd.order;
  const int* ip = a.ipool + pd.ibase;
  const void* const* cp = a.ppool + pd.pbase;
  for (int k = 0; k < pd.order; ++k) {
    x->modes[k] = y->modes[k] = ip[k];
    x->cores[k] = cp[k];
    y->cores[k] = cp[pd.order + k];
  }
  for (int k = 0; k <= pd.order; ++k) {
    x->ranks[k] = ip[pd.order + k];
    y->ranks[k] = ip[2 * pd.order + 1 + k];
  }
  *jout = pd.jout;
}

// NT: workgroup size the kernel is compiled for (256: one wave per SIMD with
// the full register file; 512: two waves per SIMD).
template <typename Tin, int NT>
__global__ __launch_bounds__(NT) void batch_kernel(BatchArgs a) {
  typedef float Tc;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double red[16];
  __shared__ TTDev sx, sy;
  __shared__ Tc one[1];
  if (threadIdx.x == 0) one[0] = 1.f;
  Tc* lds = reinterpret_cast<Tc*>(smem);
  Tc* ig = reinterpret_cast<Tc*>(a.iface) + (long)blockIdx.x * a.iface_stride;
  const int beg = a.wg_begin[blockIdx.x], end = a.wg_begin[blockIdx.x + 1];
  for (int w = beg; w < end; ++w) {
    const int p = a.order[w];
    long jout;
    if (threadIdx.x == 0) load_pair<Tin>(a, p, &sx, &sy, &jout);
    __syncthreads();
    jout = a.pairs[p].jout;
    const int N = sx.order;
    // interfaces in LDS when both fit, else in this workgroup's slice
    int mrp = 1;
    for (int b = 1; b <= N; ++b) mrp = max(mrp, sx.ranks[b] * iface_pitch(sy.ranks[b]));
    Tc* bufA = (2 * mrp <= a.lds_elems) ? lds : ig;
    Tc* bufB = bufA + mrp;
    if (threadIdx.x == 0) bufA[0] = 1.f;
    __syncthreads();
    Tc* cur = bufA;
    Tc* nxt = bufB;
    for (int k = N - 1; k >= 1; --k) {
      rl_step_chain<Tin, Tc>(sx, sy, k, cur, iface_pitch(sy.ranks[k + 1]), nxt, iface_pitch(sy.ranks[k]));
      Tc* t = cur;
      cur = nxt;
      nxt = t;
      if (k == N - 2 && (a.ops & TTC_OP_SUFFIX2)) {
        const int R = sx.ranks[k], P = sy.ranks[k], ld = iface_pitch(P);
        for (int e = threadIdx.x; e < R * P; e += blockDim.x) a.junction[jout + e] = cur[(e / P) * ld + (e % P)];
      }
    }
    if (a.ops & TTC_OP_INNER) {
      // W_1 = sum_i G_x^(0)[0, i, :]^T G_y^(0)[0, i, :] into the free buffer
      // (from W_0 = [1]), then the FP64 meet with V_1 held in `cur`.
      lr_step_chain<Tin, Tc>(sx, sy, 0, one, 1, nxt, iface_pitch(sy.ranks[1]));
      const int R1 = sx.ranks[1], P1 = sy.ranks[1], ld = iface_pitch(P1);
      double acc = 0.0;
      for (int e = threadIdx.x; e < R1 * P1; e += blockDim.x) {
        const int o = (e / P1) * ld + (e % P1);
        acc += (double)nxt[o] * (double)cur[o];
      }
      acc = wg_sum_f64(acc, red);
      if (threadIdx.x == 0) a.inner[p] = acc;
    }
    __syncthreads();
  }
}

hipError_t batch_set_lds(int bytes) {
  const void* ks[] = {reinterpret_cast<const void*>(&batch_kernel<float, 256>),
                      reinterpret_cast<const void*>(&batch_kernel<float, 512>),
                      reinterpret_cast<const void*>(&batch_kernel<bf16_t, 256>),
                      reinterpret_cast<const void*>(&batch_kernel<bf16_t, 512>)};
  for (const void* k : ks) {
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_batch(ttc_dtype dt, const BatchArgs& a, int grid, int threads, hipStream_t s) {
  const size_t lds = (size_t)a.lds_elems * sizeof(float);
  if (dt == TTC_BF16) {
    if (threads <= 256) hipLaunchKernelGGL((batch_kernel<bf16_t, 256>), dim3(grid), dim3(256), lds, s, a);
    else hipLaunchKernelGGL((batch_kernel<bf16_t, 512>), dim3(grid), dim3(512), lds, s, a);
  } else {
    if (threads <= 256) hipLaunchKernelGGL((batch_kernel<float, 256>), dim3(grid), dim3(256), lds, s, a);
    else hipLaunchKernelGGL((batch_kernel<float, 512>), dim3(grid), dim3(512), lds, s, a);
  }
  return hipGetLastError();
}

}  // namespace ttc
