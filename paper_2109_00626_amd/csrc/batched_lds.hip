// Batched interface sweeps with both interfaces of a pair held in LDS.
//
// Persistent launch: each workgroup owns a list of pairs fixed by the host
// planner (longest first onto the least-loaded workgroup), no device-side
// queue and no atomics.  For a pair of order N the workgroup sweeps right to
// left from V_N = [1] with the LDS-resident steps of sweep_lds.hpp (each
// step in its cheaper contraction order, the interface written in the
// layout the next step reads), stores V_{N-2} (the junction of the
// contraction over the last two positions) when asked, and finishes
// <X, Y> = sum_i G_x^(0)[0, i, :] V_1 G_y^(0)[0, i, :]^T with an MFMA
// product and an FP64 reduction.  Two interface buffers of `buf_elems`
// floats each make up the dynamic LDS.
#include "sweep_lds.hpp"
#include "ttc_batch.h"
#include "ttc_device.hpp"

namespace ttc {

template <typename Tin, int NT>
__global__ __launch_bounds__(NT) void batch_lds_kernel(BatchArgs a) {
  constexpr int NW = NT / 64;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double red[16];
  __shared__ TTDev sx, sy;
  TTC_LDS float* const buf0 = (TTC_LDS float*)(smem);
  TTC_LDS float* const buf1 = buf0 + a.buf_elems;
  const int beg = a.wg_begin[blockIdx.x], end = a.wg_begin[blockIdx.x + 1];
  for (int w = beg; w < end; ++w) {
    const int p = a.order[w];
    if (threadIdx.x == 0) {
      const PairDev pd = a.pairs[p];
      sx.order = sy.order = pd.order;
      const int* ip = a.ipool + pd.ibase;
      const void* const* cp = a.ppool + pd.pbase;
      for (int k = 0; k < pd.order; ++k) {
        sx.modes[k] = sy.modes[k] = ip[k];
        sx.cores[k] = cp[k];
        sy.cores[k] = cp[pd.order + k];
      }
      for (int k = 0; k <= pd.order; ++k) {
        sx.ranks[k] = ip[pd.order + k];
        sy.ranks[k] = ip[2 * pd.order + 1 + k];
      }
    }
    // V_N = [1], padded to a 16 x 16 block (pitch lds_pitch(1))
    for (int e = threadIdx.x; e < 16 * lds_pitch(1); e += NT) buf0[e] = (e == 0) ? 1.f : 0.f;
    __syncthreads();
    const int N = sx.order;
    TTC_LDS float* in = buf0;
    TTC_LDS float* out = buf1;
    bool yf = step_y_first(sx.ranks[N - 1], sx.ranks[N], sy.ranks[N - 1], sy.ranks[N]);
    for (int k = N - 1; k >= 1; --k) {
      // the final product reads V_1 in the x-first (transposed) layout
      const bool yf_next = (k == 1) ? false : step_y_first(sx.ranks[k - 1], sx.ranks[k], sy.ranks[k - 1], sy.ranks[k]);
      StepOp op;
      op.I = sx.modes[k];
      if (yf) {
        op.ga = sy.cores[k];
        op.gb = sx.cores[k];
        op.Ma = sy.ranks[k];
        op.Ka = sy.ranks[k + 1];
        op.Nb = sx.ranks[k];
        op.Kb = sx.ranks[k + 1];
      } else {
        op.ga = sx.cores[k];
        op.gb = sy.cores[k];
        op.Ma = sx.ranks[k];
        op.Ka = sx.ranks[k + 1];
        op.Nb = sy.ranks[k];
        op.Kb = sy.ranks[k + 1];
      }
      lds_step<Tin, NW>(op, in, out, yf == yf_next);
      if (k == N - 2 && (a.ops & TTC_OP_SUFFIX2)) {
        // V_{N-2} (R x P) in the layout chosen for the next step
        const int R = sx.ranks[k], P = sy.ranks[k];
        const long jo = a.pairs[p].jout;
        const int tp = lds_pitch(R), np = lds_pitch(P);
        for (int e = threadIdx.x; e < R * P; e += NT) {
          const int r = e / P, c = e - r * P;
          a.junction[jo + e] = yf_next ? out[r * np + c] : out[c * tp + r];
        }
      }
      TTC_LDS float* t = in;
      in = out;
      out = t;
      yf = yf_next;
    }
    if (a.ops & TTC_OP_INNER) {
      double s = lds_final<Tin, NW>(sx.cores[0], sy.cores[0], sx.modes[0], sx.ranks[1], sy.ranks[1], in);
      s = wg_sum_f64(s, red);
      if (threadIdx.x == 0) a.inner[p] = s;
    }
    __syncthreads();
  }
}

hipError_t batch_lds_set_lds(int bytes) {
  const void* ks[] = {reinterpret_cast<const void*>(&batch_lds_kernel<float, 256>),
                      reinterpret_cast<const void*>(&batch_lds_kernel<float, 512>),
                      reinterpret_cast<const void*>(&batch_lds_kernel<bf16_t, 256>),
                      reinterpret_cast<const void*>(&batch_lds_kernel<bf16_t, 512>)};
  for (const void* k : ks) {
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_batch_lds(ttc_dtype dt, const BatchArgs& a, int grid, int threads, hipStream_t s) {
  const size_t lds = (size_t)2 * a.buf_elems * sizeof(float);
  if (dt == TTC_BF16) {
    if (threads <= 256) hipLaunchKernelGGL((batch_lds_kernel<bf16_t, 256>), dim3(grid), dim3(256), lds, s, a);
    else hipLaunchKernelGGL((batch_lds_kernel<bf16_t, 512>), dim3(grid), dim3(512), lds, s, a);
  } else {
    if (threads <= 256) hipLaunchKernelGGL((batch_lds_kernel<float, 256>), dim3(grid), dim3(256), lds, s, a);
    else hipLaunchKernelGGL((batch_lds_kernel<float, 512>), dim3(grid), dim3(512), lds, s, a);
  }
  return hipGetLastError();
}

}  // namespace ttc
