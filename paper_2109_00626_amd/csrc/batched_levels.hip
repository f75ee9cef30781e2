// Batched sweeps, level by level: launch l computes step k = N - l of every
// pair whose order allows it, one 4-wave workgroup per (pair, 16-row tile of
// V_k).  Thousands of independent workgroups per launch let the GPU overlap
// the core reads of many pairs (the sweep of one pair alone cannot hide HBM
// latency), and the launch boundary is the only synchronisation between
// steps, so the interfaces need no device-side flags or cache maintenance.
// All launches of one run are replayed from a single HIP graph.
//
// Within a workgroup the four waves split the mode index i of the step
// (i = s, s + 4, ...), each running the chained-MFMA tile of
// sweep_steps.hpp with V_{k+1} read from the pair's interface buffer in
// global memory; the four partial tiles are summed in LDS in a fixed order.
// The last launch forms W_1 from the first cores and the FP64 inner product
// sum W_1 .* V_1 per pair.
#include "sweep_steps.hpp"
#include "ttc_batch.h"
#include "ttc_device.hpp"

namespace ttc {

__device__ __forceinline__ void load_pair_desc(const LevelArgs& a, int p, TTDev* x, TTDev* y) {
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
}

template <typename Tin>
__global__ __launch_bounds__(256, 1) void level_kernel(LevelArgs a) {
  typedef float Tc;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ TTDev sx, sy;
  const LevelItem it = a.items[blockIdx.x];
  if (threadIdx.x == 0) load_pair_desc(a, it.pair, &sx, &sy);
  __syncthreads();
  const int p = it.pair, rt = it.rt;
  const int N = sx.order, k = N - a.level;
  const int Rp = sx.ranks[k], Pp = sy.ranks[k], Pn = sy.ranks[k + 1];
  const long cap = a.vcap[p];
  Tc* base = a.vbuf + a.voff[p];
  const Tc* Vin = (k == N - 1) ? a.one : base + ((a.level + 1) & 1) * cap;
  Tc* Vout = base + (a.level & 1) * cap;
  const int w = threadIdx.x >> 6;
  typename Mfma<Tc>::acc acc[SW_MAXT];
  typedef typename Mfma<Tc>::acc acc_t;
#pragma unroll
  for (int t = 0; t < SW_MAXT; ++t) acc[t] = acc_t{0, 0, 0, 0};
  rl_tile_v<Tin, Tc>(sx, sy, k, gptr<Tc>(Vin), (k == N - 1) ? 1 : Pn, rt, w, 4, acc);
  // partial tiles of the 4 waves -> LDS -> fixed-order sum
  Tc* red = reinterpret_cast<Tc*>(smem);  // [4][16][Pp]
  const int PT = (Pp + 15) >> 4;
  const int lane = threadIdx.x & 63, li = lane & 15, g = lane >> 4;
#pragma unroll
  for (int t = 0; t < SW_MAXT; ++t) {
    if (t < PT) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int rr = Mfma<Tc>::row(g, v), pp = t * 16 + li;
        if (pp < Pp) red[(w * 16 + rr) * Pp + pp] = acc[t][v];
      }
    }
  }
  __syncthreads();
  const int rows = min(16, Rp - rt * 16);
  const bool junc = (a.ops & TTC_OP_SUFFIX2) && k == N - 2;
  for (int e = threadIdx.x; e < rows * Pp; e += blockDim.x) {
    const Tc v = red[e] + red[16 * Pp + e] + red[32 * Pp + e] + red[48 * Pp + e];
    const int r = rt * 16 + e / Pp, c = e % Pp;
    Vout[r * Pp + c] = v;
    if (junc) a.junction[a.pairs[p].jout + r * Pp + c] = v;
  }
}

// W_1 = sum_i G_x^(0)[0, i, :]^T G_y^(0)[0, i, :], then <X, Y> = sum W_1 .* V_1 (FP64).
template <typename Tin>
__global__ __launch_bounds__(256) void meet_level_kernel(LevelArgs a) {
  typedef float Tc;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ TTDev sx, sy;
  __shared__ double red[16];
  const int p = a.items[blockIdx.x].pair;
  if (threadIdx.x == 0) load_pair_desc(a, p, &sx, &sy);
  __syncthreads();
  const int N = sx.order;
  const int I = sx.modes[0], R1 = sx.ranks[1], P1 = sy.ranks[1];
  Tc* W1 = reinterpret_cast<Tc*>(smem);
  const Tin* Gx = reinterpret_cast<const Tin*>(sx.cores[0]);
  const Tin* Gy = reinterpret_cast<const Tin*>(sy.cores[0]);
  wg_gemm<Tc, Tin, Tin, Tc>(R1, P1, I, 1, 1, mv<Tin>(Gx, 1, R1), mv<Tin>(Gy, P1, 1), ov<Tc>(W1, P1, 1), false);
  __syncthreads();
  // V_1 was written by the launch of level N - 1
  const Tc* V1 = a.vbuf + a.voff[p] + ((N - 1) & 1) * a.vcap[p];
  double s = 0.0;
  for (int e = threadIdx.x; e < R1 * P1; e += blockDim.x) s += (double)W1[e] * (double)V1[e];
  s = wg_sum_f64(s, red);
  if (threadIdx.x == 0) a.inner[p] = s;
}

hipError_t level_set_lds(int level_bytes, int meet_bytes) {
  const void* lk[] = {reinterpret_cast<const void*>(&level_kernel<float>),
                      reinterpret_cast<const void*>(&level_kernel<bf16_t>)};
  for (const void* k : lk) {
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, level_bytes);
    if (e != hipSuccess) return e;
  }
  const void* mk[] = {reinterpret_cast<const void*>(&meet_level_kernel<float>),
                      reinterpret_cast<const void*>(&meet_level_kernel<bf16_t>)};
  for (const void* k : mk) {
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, meet_bytes);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_level(ttc_dtype dt, const LevelArgs& a, int nitems, size_t lds, hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  if (dt == TTC_BF16)
    hipLaunchKernelGGL(level_kernel<bf16_t>, dim3(nitems), dim3(256), lds, s, a);
  else
    hipLaunchKernelGGL(level_kernel<float>, dim3(nitems), dim3(256), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_meet_level(ttc_dtype dt, const LevelArgs& a, int npairs, size_t lds, hipStream_t s) {
  if (npairs <= 0) return hipSuccess;
  if (dt == TTC_BF16)
    hipLaunchKernelGGL(meet_level_kernel<bf16_t>, dim3(npairs), dim3(256), lds, s, a);
  else
    hipLaunchKernelGGL(meet_level_kernel<float>, dim3(npairs), dim3(256), lds, s, a);
  return hipGetLastError();
}

}  // namespace ttc
