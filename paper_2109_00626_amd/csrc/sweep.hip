// Interface sweeps over TT cores (inner products, shared-block partial
// contractions, and the inner product's gradient).
//
// Left to right (the paper's K = A_x^T A_y generalised, Section III):
//   W_{k+1} = sum_i G_x^(k)[:, i, :]^T W_k G_y^(k)[:, i, :]
// computed per chunk of i as two MFMA products:
//   T(R_k x (i, P_{k+1}))   = W_k (R_k x P_k) . G_y^(k)[:, i, :]   (G_y viewed row-major)
//   W_{k+1}(R_{k+1} x P_{k+1}) += sum_i G_x^(k)[:, i, :]^T . T_i
// Right to left:
//   V_k = sum_i G_x^(k)[:, i, :] V_{k+1} G_y^(k)[:, i, :]^T
//   S_i = G_x^(k)[:, i, :] . V_{k+1};  V_k += sum_i S_i . G_y^(k)[:, i, :]^T
// Interfaces and the per-mode intermediate live in LDS when they fit,
// otherwise in a per-block slice of the caller's workspace.
#include "sweep_steps.hpp"
#include "ttc_device.hpp"
#include "ttc_internal.h"

namespace ttc {

template <typename Tin>
__device__ __forceinline__ const Tin* core_ptr(const TTDev& t, int k) {
  return reinterpret_cast<const Tin*>(t.cores[k]);
}

// W_{k+1} from W_k (both in `Wp`/`Wn`, row-major).
template <typename Tin, typename Tc>
__device__ void lr_step(const TTDev& x, const TTDev& y, int k, const Tc* Wp, Tc* Wn, Tc* T, int tcap) {
  const int Rp = x.ranks[k], Rn = x.ranks[k + 1];
  const int Pp = y.ranks[k], Pn = y.ranks[k + 1];
  const int I = x.modes[k];
  const Tin* Gx = core_ptr<Tin>(x, k);
  const Tin* Gy = core_ptr<Tin>(y, k);
  int ic = tcap / (Rp * Pn);
  ic = ic < 1 ? 1 : (ic > I ? I : ic);
  for (int i0 = 0; i0 < I; i0 += ic) {
    const int icn = (I - i0) < ic ? (I - i0) : ic;
    // T[r'][(ii, p)] = sum_p' W[r'][p'] Gy[p'][i0 + ii][p]
    wg_gemm<Tc, Tc, Tin, Tc>(Rp, icn * Pn, Pp, 1, 1, mv<Tc>(Wp, Pp, 1), mv<Tin>(Gy + (long)i0 * Pn, I * Pn, 1),
                             ov<Tc>(T, icn * Pn, 1), false);
    __syncthreads();
    // Wn[r][p] += sum_ii sum_r' Gx[r'][i0 + ii][r] T[r'][ii][p]
    wg_gemm<Tc, Tin, Tc, Tc>(Rn, Pn, Rp, 1, icn, mv<Tin>(Gx + (long)i0 * Rn, 1, I * Rn, Rn),
                             mv<Tc>(T, icn * Pn, 1, Pn), ov<Tc>(Wn, Pn, 1), i0 > 0);
    __syncthreads();
  }
}

// V_k from V_{k+1}.
template <typename Tin, typename Tc>
__device__ void rl_step(const TTDev& x, const TTDev& y, int k, const Tc* Vn, Tc* Vp, Tc* T, int tcap) {
  const int Rp = x.ranks[k], Rn = x.ranks[k + 1];
  const int Pp = y.ranks[k], Pn = y.ranks[k + 1];
  const int I = x.modes[k];
  const Tin* Gx = core_ptr<Tin>(x, k);
  const Tin* Gy = core_ptr<Tin>(y, k);
  int ic = tcap / (Rp * Pn);
  ic = ic < 1 ? 1 : (ic > I ? I : ic);
  for (int i0 = 0; i0 < I; i0 += ic) {
    const int icn = (I - i0) < ic ? (I - i0) : ic;
    // S[ii][r][p'] = sum_r' Gx[r][i0 + ii][r'] V[r'][p']
    wg_gemm<Tc, Tin, Tc, Tc>(Rp, Pn, Rn, icn, 1, mv<Tin>(Gx + (long)i0 * Rn, I * Rn, 1, 0, Rn), mv<Tc>(Vn, Pn, 1),
                             ov<Tc>(T, Pn, 1, Rp * Pn), false);
    __syncthreads();
    // Vp[r][p] += sum_ii sum_p' S[ii][r][p'] Gy[p][i0 + ii][p']
    wg_gemm<Tc, Tc, Tin, Tc>(Rp, Pp, Pn, 1, icn, mv<Tc>(T, Pn, 1, Rp * Pn),
                             mv<Tin>(Gy + (long)i0 * Pn, 1, I * Pn, Pn), ov<Tc>(Vp, Pp, 1), i0 > 0);
    __syncthreads();
  }
}

template <typename Tc>
__device__ void wg_copy(Tc* dst, const Tc* src, int n) {
  for (int e = threadIdx.x; e < n; e += blockDim.x) dst[e] = src[e];
}

// Runs a sweep in `dir` and returns the buffer that holds the final interface.
template <typename Tin, typename Tc>
__device__ Tc* run_sweep(const TTDev& x, const TTDev& y, int dir, int stop, Tc* bufA, Tc* bufB, Tc* T,
                         int tcap) {
  if (threadIdx.x == 0) bufA[0] = (Tc)1;
  __syncthreads();
  Tc* cur = bufA;
  Tc* nxt = bufB;
  if (dir == 0) {
    for (int k = 0; k < stop; ++k) {
      lr_step<Tin, Tc>(x, y, k, cur, nxt, T, tcap);
      Tc* t = cur;
      cur = nxt;
      nxt = t;
    }
  } else {
    for (int k = x.order - 1; k >= stop; --k) {
      rl_step<Tin, Tc>(x, y, k, cur, nxt, T, tcap);
      Tc* t = cur;
      cur = nxt;
      nxt = t;
    }
  }
  return cur;
}

// Chained-MFMA sweep (ranks <= 128); interfaces use the odd-pitch layout.
template <typename Tin, typename Tc>
__device__ Tc* run_sweep_chain(const TTDev& x, const TTDev& y, int dir, int stop, Tc* bufA, Tc* bufB) {
  if (threadIdx.x == 0) bufA[0] = (Tc)1;
  __syncthreads();
  Tc* cur = bufA;
  Tc* nxt = bufB;
  if (dir == 0) {
    for (int k = 0; k < stop; ++k) {
      lr_step_chain<Tin, Tc>(x, y, k, cur, iface_pitch(y.ranks[k]), nxt, iface_pitch(y.ranks[k + 1]));
      Tc* t = cur;
      cur = nxt;
      nxt = t;
    }
  } else {
    for (int k = x.order - 1; k >= stop; --k) {
      rl_step_chain<Tin, Tc>(x, y, k, cur, iface_pitch(y.ranks[k + 1]), nxt, iface_pitch(y.ranks[k]));
      Tc* t = cur;
      cur = nxt;
      nxt = t;
    }
  }
  return cur;
}

template <typename Tin, typename Tc>
__global__ __launch_bounds__(256) void sweep_kernel(SweepArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int b = blockIdx.x;
  const int dir = a.dir[b];
  if (dir < 0) return;
  Tc* bufA = a.i_global ? reinterpret_cast<Tc*>(a.i_global) + b * a.i_stride : reinterpret_cast<Tc*>(smem);
  Tc* bufB = bufA + a.max_rp;
  const int stop = a.stop[b];
  const int R = a.x.ranks[stop], P = a.y.ranks[stop];
  Tc* out = reinterpret_cast<Tc*>(a.out[b]);
  if (a.chain) {
    Tc* res = run_sweep_chain<Tin, Tc>(a.x, a.y, dir, stop, bufA, bufB);
    const int ld = iface_pitch(P);
    for (int e = threadIdx.x; e < R * P; e += blockDim.x) out[e] = res[(e / P) * ld + (e % P)];
    return;
  }
  Tc* lds_free = a.i_global ? reinterpret_cast<Tc*>(smem) : bufB + a.max_rp;
  Tc* T = a.t_global ? reinterpret_cast<Tc*>(a.t_global) + b * a.t_stride : lds_free;
  Tc* res = run_sweep<Tin, Tc>(a.x, a.y, dir, stop, bufA, bufB, T, a.tcap);
  wg_copy<Tc>(out, res, R * P);
}

// z = sum W .* V, products and sum in FP64 (deterministic tree).
template <typename Tc>
__global__ __launch_bounds__(256) void meet_kernel(const Tc* W, const Tc* V, int n, double* out) {
  __shared__ double scratch[16];
  double s = 0.0;
  for (int e = threadIdx.x; e < n; e += blockDim.x) s += (double)W[e] * (double)V[e];
  s = wg_sum_f64(s, scratch);
  if (threadIdx.x == 0) out[0] = s;
}

// ------------------------------------------------------------------ gradient
// Phase A: block 0 sweeps left to right and stores W_{s c}; block 1 sweeps
// right to left and stores V_{min((s+1) c, N)}.
template <typename Tin, typename Tc>
__global__ __launch_bounds__(256) void grad_ckpt_kernel(GradArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  Tc* bufA = a.i_global ? reinterpret_cast<Tc*>(a.i_global) + blockIdx.x * a.i_stride : reinterpret_cast<Tc*>(smem);
  Tc* bufB = bufA + a.max_rp;
  Tc* lds_free = a.i_global ? reinterpret_cast<Tc*>(smem) : bufB + a.max_rp;
  Tc* T = a.t_global ? reinterpret_cast<Tc*>(a.t_global) + blockIdx.x * a.t_stride : lds_free;
  const int N = a.x.order, c = a.stride, ns = a.nseg;
  Tc* ckW = reinterpret_cast<Tc*>(a.ckW);
  Tc* ckV = reinterpret_cast<Tc*>(a.ckV);
  if (threadIdx.x == 0) bufA[0] = (Tc)1;
  __syncthreads();
  Tc* cur = bufA;
  Tc* nxt = bufB;
  if (blockIdx.x == 0) {
    for (int k = 0;; ++k) {
      if (k % c == 0) {
        wg_copy<Tc>(ckW + (long)(k / c) * a.max_rp, cur, a.x.ranks[k] * a.y.ranks[k]);
        if (k / c == ns - 1) break;
      }
      lr_step<Tin, Tc>(a.x, a.y, k, cur, nxt, T, a.tcap);
      Tc* t = cur;
      cur = nxt;
      nxt = t;
    }
  } else {
    for (int j = N;; --j) {
      // cur holds V_j
      int slot = -1;
      if (j == N) slot = ns - 1;
      else if (j % c == 0) slot = j / c - 1;
      if (slot >= 0) wg_copy<Tc>(ckV + (long)slot * a.max_rp, cur, a.x.ranks[j] * a.y.ranks[j]);
      if (slot == 0) break;
      rl_step<Tin, Tc>(a.x, a.y, j - 1, cur, nxt, T, a.tcap);
      Tc* t = cur;
      cur = nxt;
      nxt = t;
    }
  }
}

// Phase B: block s recomputes the interfaces of its segment from the
// checkpoints: V_{k+1} right to left and W_k left to right, each stored in
// slot k.
template <typename Tin, typename Tc>
__global__ __launch_bounds__(256) void grad_seg_kernel(GradArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int s = blockIdx.x;
  const int N = a.x.order, c = a.stride;
  const int k0 = s * c, k1 = (k0 + c < N) ? k0 + c : N;
  Tc* bufA = a.i_global ? reinterpret_cast<Tc*>(a.i_global) + blockIdx.x * a.i_stride : reinterpret_cast<Tc*>(smem);
  Tc* bufB = bufA + a.max_rp;
  Tc* lds_free = a.i_global ? reinterpret_cast<Tc*>(smem) : bufB + a.max_rp;
  Tc* T = a.t_global ? reinterpret_cast<Tc*>(a.t_global) + blockIdx.x * a.t_stride : lds_free;
  Tc* segV = reinterpret_cast<Tc*>(a.segV);
  Tc* segW = reinterpret_cast<Tc*>(a.segW);
  const Tc* ckW = reinterpret_cast<const Tc*>(a.ckW) + (long)s * a.max_rp;
  const Tc* ckV = reinterpret_cast<const Tc*>(a.ckV) + (long)s * a.max_rp;
  // right interfaces V_{k1} .. V_{k0 + 1}
  wg_copy<Tc>(segV + (long)(k1 - 1) * a.max_rp, ckV, a.x.ranks[k1] * a.y.ranks[k1]);
  __syncthreads();
  for (int k = k1 - 1; k > k0; --k) {
    rl_step<Tin, Tc>(a.x, a.y, k, segV + (long)k * a.max_rp, segV + (long)(k - 1) * a.max_rp, T, a.tcap);
  }
  // left interfaces W_{k0} .. W_{k1 - 1}
  wg_copy<Tc>(bufA, ckW, a.x.ranks[k0] * a.y.ranks[k0]);
  __syncthreads();
  Tc* cur = bufA;
  Tc* nxt = bufB;
  for (int k = k0; k < k1; ++k) {
    wg_copy<Tc>(segW + (long)k * a.max_rp, cur, a.x.ranks[k] * a.y.ranks[k]);
    if (k + 1 < k1) {
      lr_step<Tin, Tc>(a.x, a.y, k, cur, nxt, T, a.tcap);
      Tc* t = cur;
      cur = nxt;
      nxt = t;
    }
    __syncthreads();
  }
}

// Phase C: block (t, k, i) writes the gradient slice of core k at mode
// index i (t = 0: X, t = 1: Y) from W_k and V_{k+1}:
//   dX_k[:, i, :] = gz W_k G_y^(k)[:, i, :] V_{k+1}^T,
//   dY_k[:, i, :] = gz W_k^T G_x^(k)[:, i, :] V_{k+1}.
// Every slice is independent, so the whole gradient is one wide launch.
template <typename Tin, typename Tc>
__global__ __launch_bounds__(256) void grad_core_kernel(GradArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int N = a.x.order;
  const int t = blockIdx.x & 1, rest = blockIdx.x >> 1;
  const int k = rest % N, i = rest / N;
  const int I = a.x.modes[k];
  if (i >= I) return;
  void* outp = t == 0 ? a.dx[k] : a.dy[k];
  if (!outp) return;
  const int Rp = a.x.ranks[k], Rn = a.x.ranks[k + 1];
  const int Pp = a.y.ranks[k], Pn = a.y.ranks[k + 1];
  const Tc* W = reinterpret_cast<const Tc*>(a.segW) + (long)k * a.max_rp;  // Rp x Pp
  const Tc* V = reinterpret_cast<const Tc*>(a.segV) + (long)k * a.max_rp;  // Rn x Pn
  Tc* T = a.g_global ? reinterpret_cast<Tc*>(a.g_global) + blockIdx.x * a.g_stride : reinterpret_cast<Tc*>(smem);
  const Tc gz = (Tc)a.gz[0];
  if (t == 0) {
    const Tin* Gy = core_ptr<Tin>(a.y, k);
    Tc* dX = reinterpret_cast<Tc*>(outp);
    // T[r][p'] = sum_p W[r][p] G_y[p][i][p']
    wg_gemm<Tc, Tc, Tin, Tc>(Rp, Pn, Pp, 1, 1, mv<Tc>(W, Pp, 1), mv<Tin>(Gy + (long)i * Pn, I * Pn, 1),
                             ov<Tc>(T, Pn, 1), false);
    __syncthreads();
    // dX[r][i][r'] = gz sum_p' T[r][p'] V[r'][p']
    wg_gemm<Tc, Tc, Tc, Tc>(Rp, Rn, Pn, 1, 1, mv<Tc>(T, Pn, 1), mv<Tc>(V, 1, Pn), ov<Tc>(dX + (long)i * Rn, I * Rn, 1),
                            false, gz);
  } else {
    const Tin* Gx = core_ptr<Tin>(a.x, k);
    Tc* dY = reinterpret_cast<Tc*>(outp);
    // U[r][p'] = sum_r' G_x[r][i][r'] V[r'][p']
    wg_gemm<Tc, Tin, Tc, Tc>(Rp, Pn, Rn, 1, 1, mv<Tin>(Gx + (long)i * Rn, I * Rn, 1), mv<Tc>(V, Pn, 1),
                             ov<Tc>(T, Pn, 1), false);
    __syncthreads();
    // dY[p][i][p'] = gz sum_r W[r][p] U[r][p']
    wg_gemm<Tc, Tc, Tc, Tc>(Pp, Pn, Rp, 1, 1, mv<Tc>(W, 1, Pp), mv<Tc>(T, Pn, 1), ov<Tc>(dY + (long)i * Pn, I * Pn, 1),
                            false, gz);
  }
}

// ------------------------------------------------------------------ launchers
template <typename Tin, typename Tc>
static hipError_t set_lds(int bytes) {
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&sweep_kernel<Tin, Tc>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute(reinterpret_cast<const void*>(&grad_ckpt_kernel<Tin, Tc>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute(reinterpret_cast<const void*>(&grad_core_kernel<Tin, Tc>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&grad_seg_kernel<Tin, Tc>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

int lds_limit_bytes() { return 160 * 1024; }

hipError_t sweep_set_lds_limits() {
  hipError_t e = set_lds<double, double>(lds_limit_bytes());
  if (e != hipSuccess) return e;
  e = set_lds<float, float>(lds_limit_bytes());
  if (e != hipSuccess) return e;
  return set_lds<bf16_t, float>(lds_limit_bytes());
}

hipError_t launch_sweep(ttc_dtype dt, const SweepArgs& a, int nblocks, size_t lds, hipStream_t s) {
  switch (dt) {
    case TTC_F64: hipLaunchKernelGGL((sweep_kernel<double, double>), dim3(nblocks), dim3(256), lds, s, a); break;
    case TTC_F32: hipLaunchKernelGGL((sweep_kernel<float, float>), dim3(nblocks), dim3(256), lds, s, a); break;
    default: hipLaunchKernelGGL((sweep_kernel<bf16_t, float>), dim3(nblocks), dim3(256), lds, s, a); break;
  }
  return hipGetLastError();
}

hipError_t launch_meet(ttc_dtype dt, const void* W, const void* V, int n, double* out, hipStream_t s) {
  if (dt == TTC_F64)
    hipLaunchKernelGGL((meet_kernel<double>), dim3(1), dim3(256), 0, s, (const double*)W, (const double*)V, n, out);
  else
    hipLaunchKernelGGL((meet_kernel<float>), dim3(1), dim3(256), 0, s, (const float*)W, (const float*)V, n, out);
  return hipGetLastError();
}

hipError_t launch_grad_ckpt(ttc_dtype dt, const GradArgs& a, size_t lds, hipStream_t s) {
  switch (dt) {
    case TTC_F64: hipLaunchKernelGGL((grad_ckpt_kernel<double, double>), dim3(2), dim3(256), lds, s, a); break;
    case TTC_F32: hipLaunchKernelGGL((grad_ckpt_kernel<float, float>), dim3(2), dim3(256), lds, s, a); break;
    default: hipLaunchKernelGGL((grad_ckpt_kernel<bf16_t, float>), dim3(2), dim3(256), lds, s, a); break;
  }
  return hipGetLastError();
}

hipError_t launch_grad_core(ttc_dtype dt, const GradArgs& a, int blocks, size_t lds, hipStream_t s) {
  switch (dt) {
    case TTC_F64: hipLaunchKernelGGL((grad_core_kernel<double, double>), dim3(blocks), dim3(256), lds, s, a); break;
    case TTC_F32: hipLaunchKernelGGL((grad_core_kernel<float, float>), dim3(blocks), dim3(256), lds, s, a); break;
    default: hipLaunchKernelGGL((grad_core_kernel<bf16_t, float>), dim3(blocks), dim3(256), lds, s, a); break;
  }
  return hipGetLastError();
}

hipError_t launch_grad_seg(ttc_dtype dt, const GradArgs& a, size_t lds, hipStream_t s) {
  switch (dt) {
    case TTC_F64: hipLaunchKernelGGL((grad_seg_kernel<double, double>), dim3(a.nseg), dim3(256), lds, s, a); break;
    case TTC_F32: hipLaunchKernelGGL((grad_seg_kernel<float, float>), dim3(a.nseg), dim3(256), lds, s, a); break;
    default: hipLaunchKernelGGL((grad_seg_kernel<bf16_t, float>), dim3(a.nseg), dim3(256), lds, s, a); break;
  }
  return hipGetLastError();
}

}  // namespace ttc
