// Single-pair interface sweeps on the LDS-resident step of the batched
// kernel (sweep_lds.hpp): the interface stays in LDS for the whole sweep, each
// step in its cheaper contraction order, cores streamed from HBM.  Used for
// the inner product, the junction of a prefix or suffix contraction and the
// interfaces of the inner-product gradient when the pair qualifies (FP32 or
// BF16 cores, ranks <= 128).  M16 (BF16 cores, precision BF16): the steps of
// sweep_lds16.hpp on BF16 MFMA, the interface held as BF16 hi / lo planes.  Left-to-right sweeps run as right-to-left
// sweeps of the reversed pair with rank-transposed cores: the step
//   sum_i G_x[:, i, :]^T W G_y[:, i, :]
// of a left-to-right sweep is the right-to-left step on cores G'[a, i, b] =
// G[b, i, a].
#include "sweep_lds16.hpp"
#include "ttc_device.hpp"
#include "ttc_internal.h"

namespace ttc {

namespace {

// The interface after the step on core k, in LDS: transposed (rows p,
// pitch lds_pitch(R)) when the next step runs x first, else plain (rows r,
// pitch lds_pitch(P)); written out plain, R x P row-major.
__device__ __forceinline__ void store_iface(float* dst, const TTC_LDS float* buf, int R, int P, bool plain) {
  const int tp = lds_pitch(R), np = lds_pitch(P);
  for (int e = threadIdx.x; e < R * P; e += blockDim.x) {
    const int r = e / P, c = e - r * P;
    dst[e] = plain ? buf[r * np + c] : buf[c * tp + r];
  }
}

// The same from BF16 planes (hi at V, lo at V + lo).
__device__ __forceinline__ void store_iface16(float* dst, const TTC_LDS uint16_t* V, int lo, int R, int P,
                                              bool plain) {
  const int tp = lds16_pitch(R), np = lds16_pitch(P);
  for (int e = threadIdx.x; e < R * P; e += blockDim.x) {
    const int r = e / P, c = e - r * P;
    dst[e] = lds16_get(V, lo, plain ? r * np + c : c * tp + r);
  }
}

template <typename Tin, bool M16>
__global__ __launch_bounds__(256, 2) void pair_lds_kernel(PairLdsArgs args) {
  constexpr int NW = 4;
  static_assert(!M16 || sizeof(Tin) == 2, "BF16 MFMA steps: BF16 cores");
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double red[16];
  __shared__ TTDev sx, sy;
  const PairLdsSide& a = args.side[blockIdx.x];
  {
    const int e = threadIdx.x, N = a.x.order;
    if (e == 0) sx.order = sy.order = N;
    if (e < N) {
      sx.modes[e] = sy.modes[e] = a.x.modes[e];
      sx.cores[e] = a.x.cores[e];
      sy.cores[e] = a.y.cores[e];
    }
    if (e <= N) {
      sx.ranks[e] = a.x.ranks[e];
      sy.ranks[e] = a.y.ranks[e];
    }
  }
  TTC_LDS float* const buf = (TTC_LDS float*)smem;
  TTC_LDS uint16_t* const pl = (TTC_LDS uint16_t*)smem;  // M16: hi plane; lo plane at pl + lo
  const int lo = args.lo;
  if constexpr (M16) {
    for (int e = threadIdx.x; e < 16 * lds16_pitch(1); e += blockDim.x) {
      pl[e] = (e == 0) ? (uint16_t)0x3F80u : (uint16_t)0;
      pl[lo + e] = 0;
    }
  } else {
    for (int e = threadIdx.x; e < 16 * lds_pitch(1); e += blockDim.x) buf[e] = (e == 0) ? 1.f : 0.f;
  }
  __syncthreads();
  const int N = sx.order, stop = a.stop;
  if (a.all && threadIdx.x == 0) a.all[(long)(a.slot_a * N + a.slot_b) * a.all_stride] = 1.f;
  bool yf = step_y_first(sx.ranks[N - 1], sx.ranks[N], sy.ranks[N - 1], sy.ranks[N]);
  for (int k = N - 1; k >= stop; --k) {
    // the last interface (and the final product) read the x-first layout
    const bool yf_next = (k == stop) ? false : step_y_first(sx.ranks[k - 1], sx.ranks[k], sy.ranks[k - 1], sy.ranks[k]);
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
    if constexpr (M16) lds16_step_inplace<NW>(op, pl, lo, yf == yf_next, nullptr);
    else lds_step_inplace<Tin, NW>(op, buf, yf == yf_next);
    // (the step ends with a barrier; the next step overwrites buf only after
    // its own barrier, which every thread reaches after these stores)
    if constexpr (M16) {
      if (k == stop && a.out) store_iface16(a.out, pl, lo, sx.ranks[k], sy.ranks[k], yf_next);
    } else {
      if (a.all && k >= 1)
        store_iface(a.all + (long)(a.slot_a * k + a.slot_b) * a.all_stride, buf, sx.ranks[k], sy.ranks[k], yf_next);
      if (k == stop && a.out) store_iface(a.out, buf, sx.ranks[k], sy.ranks[k], yf_next);
    }
    yf = yf_next;
  }
  if (a.inner) {
    double s;
    if constexpr (M16) s = lds16_final<NW>(sx.cores[0], sy.cores[0], sx.modes[0], sx.ranks[1], sy.ranks[1], pl, lo);
    else s = lds_final<Tin, NW>(sx.cores[0], sy.cores[0], sx.modes[0], sx.ranks[1], sy.ranks[1], buf);
    s = wg_sum_f64(s, red);
    if (threadIdx.x == 0) *a.inner = s;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void core_reverse_kernel(CoreRevArgs a) {
  const CoreRevItem& c = a.c[blockIdx.y];
  const long n = (long)c.R * c.I * c.R1;
  const T* src = reinterpret_cast<const T*>(c.src);
  T* dst = reinterpret_cast<T*>(c.dst);
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    // e indexes the destination (R1, I, R)
    const int r = (int)(e % c.R);
    const long t = e / c.R;
    const int i = (int)(t % c.I);
    const int r1 = (int)(t / c.I);
    dst[e] = src[((long)r * c.I + i) * c.R1 + r1];
  }
}

// Floats of the one in-place interface buffer for a side; m16: elements of
// each BF16 plane (a multiple of 8, so the lo plane starts 16-byte aligned;
// two planes take as many bytes as that many floats).
int side_lds_floats(const PairLdsSide& s, bool m16) {
  int m = m16 ? 16 * lds16_pitch(1) : 16 * lds_pitch(1);
  for (int b = s.stop; b <= s.x.order; ++b)
    m = std::max(m, m16 ? lds16_iface_elems(s.x.ranks[b], s.y.ranks[b]) : lds_iface_elems(s.x.ranks[b], s.y.ranks[b]));
  return (m + 7) & ~7;
}

}  // namespace

bool pair_lds_ok(const TTDev& x, const TTDev& y) {
  for (int b = 0; b <= x.order; ++b)
    if (x.ranks[b] > 128 || y.ranks[b] > 128) return false;
  for (int k = 0; k < x.order; ++k)
    if (128.0 * x.modes[k] * 128.0 * 4.0 >= 2147483647.0) return false;  // 32-bit core byte offsets
  return true;
}

hipError_t launch_pair_lds(ttc_dtype dt, const PairLdsArgs& in, int nsides, hipStream_t s) {
  PairLdsArgs a = in;
  const bool m16 = a.m16 && dt == TTC_BF16;
  int floats = 0;
  for (int q = 0; q < nsides; ++q) floats = std::max(floats, side_lds_floats(a.side[q], m16));
  a.lo = floats;
  const int bytes = floats * (int)sizeof(float);
  static std::atomic<bool> done[kMaxDevices];
  const hipError_t e = once_per_device(done, [] {
    // the largest buffer any qualifying pair needs (ranks 128)
    const int most = std::max(lds_iface_elems(128, 128), (lds16_iface_elems(128, 128) + 7) & ~7) * (int)sizeof(float);
    hipError_t r = hipFuncSetAttribute(reinterpret_cast<const void*>(&pair_lds_kernel<float, false>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, most);
    if (r == hipSuccess)
      r = hipFuncSetAttribute(reinterpret_cast<const void*>(&pair_lds_kernel<bf16_t, false>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, most);
    if (r == hipSuccess)
      r = hipFuncSetAttribute(reinterpret_cast<const void*>(&pair_lds_kernel<bf16_t, true>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, most);
    return r;
  });
  if (e != hipSuccess) return e;
  if (m16) hipLaunchKernelGGL((pair_lds_kernel<bf16_t, true>), dim3(nsides), dim3(256), bytes, s, a);
  else if (dt == TTC_BF16) hipLaunchKernelGGL((pair_lds_kernel<bf16_t, false>), dim3(nsides), dim3(256), bytes, s, a);
  else hipLaunchKernelGGL((pair_lds_kernel<float, false>), dim3(nsides), dim3(256), bytes, s, a);
  return hipGetLastError();
}

hipError_t launch_core_reverse(const CoreRevArgs& a, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  long most = 1;
  for (int q = 0; q < a.n; ++q) most = std::max(most, (long)a.c[q].R * a.c[q].I * a.c[q].R1);
  const unsigned gx = (unsigned)std::min<long>((most + 255) / 256, 1024);
  if (a.esz == 2) hipLaunchKernelGGL((core_reverse_kernel<uint16_t>), dim3(gx, a.n), dim3(256), 0, s, a);
  else hipLaunchKernelGGL((core_reverse_kernel<uint32_t>), dim3(gx, a.n), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace ttc
