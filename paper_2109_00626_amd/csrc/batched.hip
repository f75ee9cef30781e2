// Batched interface sweeps: many independent (X, Y) pairs of uneven order,
// mode sizes and ranks in one persistent launch.
//
// Each workgroup owns a list of pairs fixed by the host planner (longest
// first onto the least-loaded workgroup), so there is no device-side queue
// and no atomic.  For a pair of order N the workgroup sweeps right to left:
//   V_N = [1],  V_k = sum_i G_x^(k)[:, i, :] V_{k+1} G_y^(k)[:, i, :]^T  (k >= 1),
// stores V_{N-2} (the junction of the contraction over the last two
// positions) when asked, then forms W_1 = sum_i G_x^(0)[0, i, :]^T G_y^(0)[0, i, :]
// and finishes <X, Y> = sum W_1 .* V_1 in FP64.  Interfaces and the
// per-mode intermediate are placed per pair: in LDS when they fit the
// workgroup's budget, else in the workgroup's slice of plan memory.
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

template <typename Tin, typename Tc>
__device__ void lr_first(const TTDev& x, const TTDev& y, Tc* W1) {
  // W_1[r][p] = sum_i Gx0[0][i][r] Gy0[0][i][p]
  const int I = x.modes[0], Rn = x.ranks[1], Pn = y.ranks[1];
  const Tin* Gx = reinterpret_cast<const Tin*>(x.cores[0]);
  const Tin* Gy = reinterpret_cast<const Tin*>(y.cores[0]);
  wg_gemm<Tc, Tin, Tin, Tc>(Rn, Pn, I, 1, 1, mv<Tin>(Gx, 1, Rn), mv<Tin>(Gy, Pn, 1), ov<Tc>(W1, Pn, 1), false);
}

template <typename Tin, typename Tc>
__device__ void rl_step_b(const TTDev& x, const TTDev& y, int k, const Tc* Vn, Tc* Vp, Tc* T, int tcap) {
  const int Rp = x.ranks[k], Rn = x.ranks[k + 1];
  const int Pp = y.ranks[k], Pn = y.ranks[k + 1];
  const int I = x.modes[k];
  const Tin* Gx = reinterpret_cast<const Tin*>(x.cores[k]);
  const Tin* Gy = reinterpret_cast<const Tin*>(y.cores[k]);
  int ic = tcap / (Rp * Pn);
  ic = ic < 1 ? 1 : (ic > I ? I : ic);
  for (int i0 = 0; i0 < I; i0 += ic) {
    const int icn = (I - i0) < ic ? (I - i0) : ic;
    wg_gemm<Tc, Tin, Tc, Tc>(Rp, Pn, Rn, icn, 1, mv<Tin>(Gx + (long)i0 * Rn, I * Rn, 1, 0, Rn), mv<Tc>(Vn, Pn, 1),
                             ov<Tc>(T, Pn, 1, Rp * Pn), false);
    __syncthreads();
    wg_gemm<Tc, Tc, Tin, Tc>(Rp, Pp, Pn, 1, icn, mv<Tc>(T, Pn, 1, Rp * Pn),
                             mv<Tin>(Gy + (long)i0 * Pn, 1, I * Pn, Pn), ov<Tc>(Vp, Pp, 1), i0 > 0);
    __syncthreads();
  }
}

template <typename Tin>
__global__ __launch_bounds__(512) void batch_kernel(BatchArgs a) {
  typedef float Tc;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double red[16];
  __shared__ TTDev sx, sy;
  Tc* lds = reinterpret_cast<Tc*>(smem);
  Tc* ig = reinterpret_cast<Tc*>(a.iface) + (long)blockIdx.x * a.iface_stride;
  Tc* tg = reinterpret_cast<Tc*>(a.tbuf) + (long)blockIdx.x * a.t_stride;
  const int beg = a.wg_begin[blockIdx.x], end = a.wg_begin[blockIdx.x + 1];
  for (int w = beg; w < end; ++w) {
    const int p = a.order[w];
    long jout;
    if (threadIdx.x == 0) load_pair<Tin>(a, p, &sx, &sy, &jout);
    __syncthreads();
    jout = a.pairs[p].jout;
    const int N = sx.order;
    // per-pair placement
    int mrp = 1, mt = 1;
    for (int b = 1; b <= N; ++b) mrp = max(mrp, sx.ranks[b] * sy.ranks[b]);
    for (int k = 1; k < N; ++k) mt = max(mt, sx.ranks[k] * sy.ranks[k + 1]);
    Tc *bufA, *bufB, *T;
    int used = 0;
    if (2 * mrp <= a.lds_elems) {
      bufA = lds;
      used = 2 * mrp;
    } else {
      bufA = ig;
    }
    bufB = bufA + mrp;
    int tcap;
    if (a.lds_elems - used >= mt) {
      T = lds + used;
      tcap = a.lds_elems - used;
    } else {
      T = tg;
      tcap = a.t_stride;
    }
    if (threadIdx.x == 0) bufA[0] = 1.f;
    __syncthreads();
    Tc* cur = bufA;
    Tc* nxt = bufB;
    for (int k = N - 1; k >= 1; --k) {
      rl_step_b<Tin, Tc>(sx, sy, k, cur, nxt, T, tcap);
      Tc* t = cur;
      cur = nxt;
      nxt = t;
      if (k == N - 2 && (a.ops & TTC_OP_SUFFIX2)) {
        const int n = sx.ranks[k] * sy.ranks[k];
        for (int e = threadIdx.x; e < n; e += blockDim.x) a.junction[jout + e] = cur[e];
      }
    }
    if (a.ops & TTC_OP_INNER) {
      // W_1 into the free interface buffer, then the FP64 meet with V_1
      lr_first<Tin, Tc>(sx, sy, nxt);
      __syncthreads();
      const int n = sx.ranks[1] * sy.ranks[1];
      double s = 0.0;
      for (int e = threadIdx.x; e < n; e += blockDim.x) s += (double)nxt[e] * (double)cur[e];
      s = wg_sum_f64(s, red);
      if (threadIdx.x == 0) a.inner[p] = s;
    }
    __syncthreads();
  }
}

hipError_t batch_set_lds(int bytes) {
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&batch_kernel<float>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&batch_kernel<bf16_t>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

hipError_t launch_batch(ttc_dtype dt, const BatchArgs& a, int grid, int threads, hipStream_t s) {
  const size_t lds = (size_t)a.lds_elems * sizeof(float);
  if (dt == TTC_BF16)
    hipLaunchKernelGGL(batch_kernel<bf16_t>, dim3(grid), dim3(threads), lds, s, a);
  else
    hipLaunchKernelGGL(batch_kernel<float>, dim3(grid), dim3(threads), lds, s, a);
  return hipGetLastError();
}

}  // namespace ttc
