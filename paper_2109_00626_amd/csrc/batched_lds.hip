// Batched interface sweeps with both interfaces of a pair held in LDS.
//
// Persistent launch over a list of pairs sorted longest first.  Workgroups
// claim the next list position from a counter in global memory when they
// finish a pair (so the slowest pairs start first and no workgroup idles
// while work remains), or, when no counter is given, each walks a fixed
// slice of the list.  The counter is an agent-scope atomic (coherent across
// the dies' L2 caches); the last workgroup to exit clears it, so every
// launch (graph replays included) starts from zero.  Launches sharing one
// counter must not overlap.  For a pair of order N the workgroup sweeps right to
// left from V_N = [1] with the LDS-resident steps of sweep_lds.hpp (each
// step in its cheaper contraction order, the interface written in the
// layout the next step reads), stores V_{N-2} (the junction of the
// contraction over the last two positions) when asked, and finishes
// <X, Y> = sum_i G_x^(0)[0, i, :] V_1 G_y^(0)[0, i, :]^T with an MFMA
// product and an FP64 reduction.  The dynamic LDS holds two interface
// buffers of `buf_elems` floats used alternately, or (in-place variants) one
// buffer that each step overwrites: FP32, or for BF16 cores on BF16 MFMA two
// BF16 planes (hi, lo) of `buf_elems` elements each (sweep_lds16.hpp).
#include "sweep_lds16.hpp"
#include "ttc_batch.h"
#include "ttc_device.hpp"

namespace ttc {

// ONE: a single interface buffer updated in place (two workgroups per CU);
// otherwise two buffers used alternately.  M16 (BF16 cores, in place): the
// steps run on BF16 MFMA with the interface as BF16 hi / lo planes.
template <typename Tin, int NT, bool ONE, bool M16 = false>
__global__ __launch_bounds__(NT, ONE ? 2 : 1) void batch_lds_kernel(BatchArgs a) {
  constexpr int NW = NT / 64;
  static_assert(!M16 || (ONE && sizeof(Tin) == 2), "BF16 MFMA steps: BF16 cores, in place");
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double red[16];
  __shared__ TTDev sx, sy;
  TTC_LDS float* const buf0 = (TTC_LDS float*)(smem);
  TTC_LDS float* const buf1 = ONE ? buf0 : buf0 + a.buf_elems;
  TTC_LDS uint16_t* const pl = (TTC_LDS uint16_t*)(smem);  // M16: hi plane; lo plane at pl + lo
  const int lo = a.buf_elems;
  __shared__ int claimed;
  const bool dyn = a.claim != nullptr;
  const int end = dyn ? a.npairs : a.wg_begin[blockIdx.x + 1];
  for (int w = dyn ? 0 : a.wg_begin[blockIdx.x];; ++w) {
    if (dyn) {
      // every thread has read the previous value: the pair's body below
      // passes several barriers before the next claim
      if (threadIdx.x == 0) claimed = atomicAdd(a.claim, 1);
      __syncthreads();
      w = claimed;
    }
    if (w >= end) break;
    const int p = a.order[w];
    if (a.clock && threadIdx.x == 0) {
      a.clock[2 * p] = (long long)__builtin_readcyclecounter();
      a.clock[2 * a.npairs + p] = blockIdx.x;
    }
    {
      // descriptors, one entry per thread
      const PairDev pd = a.pairs[p];
      const int* ip = a.ipool + pd.ibase;
      const void* const* cp = a.ppool + pd.pbase;
      const int e = threadIdx.x, N = pd.order;
      if (e == 0) sx.order = sy.order = N;
      if (e < N) {
        sx.modes[e] = sy.modes[e] = ip[e];
        sx.cores[e] = cp[e];
        sy.cores[e] = cp[N + e];
      }
      if (e <= N) {
        sx.ranks[e] = ip[N + e];
        sy.ranks[e] = ip[2 * N + 1 + e];
      }
    }
    // V_N = [1], padded to a 16 x 16 block (pitch lds_pitch(1), or
    // lds16_pitch(1) in both planes)
    if constexpr (M16) {
      for (int e = threadIdx.x; e < 16 * lds16_pitch(1); e += NT) {
        pl[e] = (e == 0) ? (uint16_t)0x3F80u : (uint16_t)0;
        pl[lo + e] = 0;
      }
    } else {
      for (int e = threadIdx.x; e < 16 * lds_pitch(1); e += NT) buf0[e] = (e == 0) ? 1.f : 0.f;
    }
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
      if constexpr (M16) lds16_step_inplace<NW>(op, pl, lo, yf == yf_next, a.stage ? pl + 2 * lo : nullptr);
      else if constexpr (ONE) lds_step_inplace<Tin, NW>(op, in, yf == yf_next);
      else lds_step<Tin, NW>(op, in, out, yf == yf_next);
      if (k == N - 2 && (a.ops & TTC_OP_SUFFIX2)) {
        // V_{N-2} (R x P) in the layout chosen for the next step
        const int R = sx.ranks[k], P = sy.ranks[k];
        const long jo = a.pairs[p].jout;
        if constexpr (M16) {
          const int tp = lds16_pitch(R), np = lds16_pitch(P);
          for (int e = threadIdx.x; e < R * P; e += NT) {
            const int r = e / P, c = e - r * P;
            a.junction[jo + e] = lds16_get(pl, lo, yf_next ? r * np + c : c * tp + r);
          }
        } else {
          const int tp = lds_pitch(R), np = lds_pitch(P);
          for (int e = threadIdx.x; e < R * P; e += NT) {
            const int r = e / P, c = e - r * P;
            a.junction[jo + e] = yf_next ? out[r * np + c] : out[c * tp + r];
          }
        }
      }
      TTC_LDS float* t = in;
      in = out;
      out = t;
      yf = yf_next;
      if (a.clock && threadIdx.x == 0)
        a.clock[3L * a.npairs + 32L * p + (N - 1 - k)] = (long long)__builtin_readcyclecounter();
    }
    if (a.ops & TTC_OP_INNER) {
      double s;
      if constexpr (M16) s = lds16_final<NW>(sx.cores[0], sy.cores[0], sx.modes[0], sx.ranks[1], sy.ranks[1], pl, lo);
      else s = lds_final<Tin, NW>(sx.cores[0], sy.cores[0], sx.modes[0], sx.ranks[1], sy.ranks[1], in);
      s = wg_sum_f64(s, red);
      if (threadIdx.x == 0) a.inner[p] = s;
    }
    __syncthreads();
    if (a.clock && threadIdx.x == 0) {
      const long long t = (long long)__builtin_readcyclecounter();
      a.clock[2 * p + 1] = t;
      a.clock[3L * a.npairs + 32L * p + (N - 1)] = t;
    }
  }
  if (dyn && threadIdx.x == 0) {
    // every claim of this workgroup precedes its exit count; the last one
    // out finds no claims pending and clears both counters
    if (atomicAdd(a.claim + 1, 1) == (int)gridDim.x - 1) {
      atomicExch(a.claim, 0);
      atomicExch(a.claim + 1, 0);
    }
  }
}

hipError_t batch_lds_set_lds(int bytes, int stage_bytes) {
  // bytes: two interface buffers; the in-place kernels take half
  const void* two[] = {reinterpret_cast<const void*>(&batch_lds_kernel<float, 256, false>),
                       reinterpret_cast<const void*>(&batch_lds_kernel<float, 512, false>),
                       reinterpret_cast<const void*>(&batch_lds_kernel<bf16_t, 256, false>),
                       reinterpret_cast<const void*>(&batch_lds_kernel<bf16_t, 512, false>)};
  for (const void* k : two) {
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return e;
  }
  const void* one[] = {reinterpret_cast<const void*>(&batch_lds_kernel<float, 256, true>),
                       reinterpret_cast<const void*>(&batch_lds_kernel<bf16_t, 256, true>)};
  for (const void* k : one) {
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, bytes / 2);
    if (e != hipSuccess) return e;
  }
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&batch_lds_kernel<bf16_t, 256, true, true>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, bytes / 2 + stage_bytes);
}

hipError_t launch_batch_lds(ttc_dtype dt, const BatchArgs& a, int grid, int threads, int variant, hipStream_t s) {
  if (variant == kBatchLdsB16) {
    if (dt != TTC_BF16) return hipErrorInvalidValue;
    const size_t lds = (size_t)a.buf_elems * sizeof(float) + (a.stage ? kBatchStageBytes : 0);
    hipLaunchKernelGGL((batch_lds_kernel<bf16_t, 256, true, true>), dim3(grid), dim3(256), lds, s, a);
    return hipGetLastError();
  }
  if (variant == kBatchLdsInPlace) {
    const size_t lds = (size_t)a.buf_elems * sizeof(float);
    if (dt == TTC_BF16) hipLaunchKernelGGL((batch_lds_kernel<bf16_t, 256, true>), dim3(grid), dim3(256), lds, s, a);
    else hipLaunchKernelGGL((batch_lds_kernel<float, 256, true>), dim3(grid), dim3(256), lds, s, a);
    return hipGetLastError();
  }
  const size_t lds = (size_t)2 * a.buf_elems * sizeof(float);
  if (dt == TTC_BF16) {
    if (threads <= 256) hipLaunchKernelGGL((batch_lds_kernel<bf16_t, 256, false>), dim3(grid), dim3(256), lds, s, a);
    else hipLaunchKernelGGL((batch_lds_kernel<bf16_t, 512, false>), dim3(grid), dim3(512), lds, s, a);
  } else {
    if (threads <= 256) hipLaunchKernelGGL((batch_lds_kernel<float, 256, false>), dim3(grid), dim3(256), lds, s, a);
    else hipLaunchKernelGGL((batch_lds_kernel<float, 512, false>), dim3(grid), dim3(512), lds, s, a);
  }
  return hipGetLastError();
}

}  // namespace ttc
