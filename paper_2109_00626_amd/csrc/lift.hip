// Output forms of a shared-block contraction.
//
// Natural-order TT (eq. (8) mode order, Algorithm 2's final permutation
// realised on cores): the junction matrix K (kr x Q) is absorbed into the
// free core next to it and its column index q is carried through the other
// side's cores as an extra bond factor (merged index (own bond) * Q + q).
// The carried-bond cores are block-diagonal copies: almost all of their
// entries are zero, so the kernel is a pure HBM write stream.  Work is split
// into lines (one fixed row bond and mode index, d1 contiguous outputs);
// each thread writes 4 consecutive outputs with one 16-byte store, the
// block-diagonal cores without a division per output.
//
// Dense form (small cases): every output entry is the product of the core
// slices along its multi-index (eq. (9)).
#include "ttc_device.hpp"
#include "ttc_internal.h"

namespace ttc {

template <typename Tin, typename Tc>
__device__ __forceinline__ Tc lift_value(const LiftCore& c, const Tc* K, int Q, int row, int i, int col) {
  const Tin* src = reinterpret_cast<const Tin*>(c.src);
  switch (c.op) {
    case LIFT_COPY:
      return cvt<Tc>(src[((long)row * c.n + i) * c.r1 + col]);
    case LIFT_ABSORB_L: {  // dst (1, n, r1*Q); col = s*Q + q
      const int s = col / Q, q = col - s * Q;
      Tc acc = 0;
      for (int r = 0; r < c.r0; ++r) acc += K[r * Q + q] * cvt<Tc>(src[((long)r * c.n + i) * c.r1 + s]);
      return acc;
    }
    case LIFT_ABSORB_R: {  // dst (r0, n, Q); row = s, col = q
      Tc acc = 0;
      const Tin* g = src + ((long)row * c.n + i) * c.r1;
      for (int r = 0; r < c.r1; ++r) acc += cvt<Tc>(g[r]) * K[r * Q + col];
      return acc;
    }
    case LIFT_DELTA: {  // dst (r0*Q, n, r1*Q)
      const int a = row / Q, q = row - a * Q;
      const int b = col / Q, qq = col - b * Q;
      return q == qq ? cvt<Tc>(src[((long)a * c.n + i) * c.r1 + b]) : (Tc)0;
    }
    case LIFT_ABSORB_M: {  // dst (ka, n, r1*Q); row = a, col = s*Q + q, q = g*kd + d
      const int s = col / Q, q = col - s * Q;
      const int g = q / c.kd, d = q - g * c.kd;
      const Tc* T = K + ((long)row * c.kg + g) * c.r0 * c.kd + d;
      Tc acc = 0;
      for (int b = 0; b < c.r0; ++b) acc += T[(long)b * c.kd] * cvt<Tc>(src[((long)b * c.n + i) * c.r1 + s]);
      return acc;
    }
    case LIFT_DELTA_SPLIT: {  // dst (r0*Q, n, kd), src (r0, n, kg); row = y*Q + g*kd + d
      const int y = row / Q, q = row - y * Q;
      const int g = q / c.kd, d = q - g * c.kd;
      return d == col ? cvt<Tc>(src[((long)y * c.n + i) * c.r1 + g]) : (Tc)0;
    }
    default: {  // LIFT_DELTA_LAST: dst (r0*Q, n, 1), src (r0, n, Q)
      const int p = row / Q, q = row - p * Q;
      return cvt<Tc>(src[((long)p * c.n + i) * c.r1 + q]);
    }
  }
}

// One line (one row bond and mode index: d1 consecutive outputs) of core cc.
template <typename Tin, typename Tc>
__device__ __forceinline__ void lift_line(const LiftArgs& a, const LiftCore& c, int l) {
  const int row = l / c.n, i = l - row * c.n;
  const Tc* K = reinterpret_cast<const Tc*>(a.K);
  Tc* dst = reinterpret_cast<Tc*>(c.dst) + (long)l * c.d1;
  const int d1 = c.d1;
  if (sizeof(Tc) == 4 && (d1 & 3) == 0 && c.op == LIFT_DELTA && (a.Q & 3) == 0) {
    // block-diagonal copy: in line (row, i) only the columns b*Q + q hold
    // entries (row = a*Q + q); the four columns of a thread share b, so one
    // division per four outputs and at most one load
    const int ra = row / a.Q, q = row - ra * a.Q;
    const Tin* src = reinterpret_cast<const Tin*>(c.src) + ((long)ra * c.n + i) * c.r1;
    for (int j = 4 * threadIdx.x; j < d1; j += 4 * blockDim.x) {
      const int b = j / a.Q, u = q - (j - b * a.Q);
      f32x4 v = {0.f, 0.f, 0.f, 0.f};
      if (u >= 0 && u < 4) {
        const float e = (float)cvt<Tc>(src[b]);
        v[0] = u == 0 ? e : 0.f;
        v[1] = u == 1 ? e : 0.f;
        v[2] = u == 2 ? e : 0.f;
        v[3] = u == 3 ? e : 0.f;
      }
      __builtin_nontemporal_store(v, reinterpret_cast<f32x4*>(dst + j));
    }
  } else if (sizeof(Tc) == 4 && (d1 & 3) == 0) {
    for (int j = 4 * threadIdx.x; j < d1; j += 4 * blockDim.x) {
      f32x4 v;
      v[0] = (float)lift_value<Tin, Tc>(c, K, a.Q, row, i, j);
      v[1] = (float)lift_value<Tin, Tc>(c, K, a.Q, row, i, j + 1);
      v[2] = (float)lift_value<Tin, Tc>(c, K, a.Q, row, i, j + 2);
      v[3] = (float)lift_value<Tin, Tc>(c, K, a.Q, row, i, j + 3);
      __builtin_nontemporal_store(v, reinterpret_cast<f32x4*>(dst + j));
    }
  } else {
    for (int j = threadIdx.x; j < d1; j += blockDim.x) dst[j] = lift_value<Tin, Tc>(c, K, a.Q, row, i, j);
  }
}

// Workgroups walk the lines of every output core in a grid-stride loop (a
// few thousand workgroups, each writing many lines, rather than one
// workgroup per line).
template <typename Tin, typename Tc>
__global__ __launch_bounds__(256) void lift_kernel(LiftArgs a, int total_lines) {
  int cc = 0;
  for (int L = blockIdx.x; L < total_lines; L += gridDim.x) {
    while (cc + 1 < a.ncores && a.c[cc + 1].line_begin <= L) ++cc;
    lift_line<Tin, Tc>(a, a.c[cc], L - a.c[cc].line_begin);
  }
}

#define TTC_DENSE_MAXR 64

template <typename Tc>
__global__ __launch_bounds__(256) void dense_kernel(DenseArgs a) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= a.numel) return;
  int idx[TTC_MAX_ORDER];
  long rem = e;
  for (int k = a.t.order - 1; k >= 0; --k) {
    idx[k] = (int)(rem % a.t.modes[k]);
    rem /= a.t.modes[k];
  }
  Tc v[TTC_DENSE_MAXR], w[TTC_DENSE_MAXR];
  v[0] = (Tc)1;
  for (int k = 0; k < a.t.order; ++k) {
    const int r0 = a.t.ranks[k], r1 = a.t.ranks[k + 1], n = a.t.modes[k];
    const Tc* G = reinterpret_cast<const Tc*>(a.t.cores[k]);
    for (int s = 0; s < r1; ++s) {
      Tc acc = 0;
      for (int r = 0; r < r0; ++r) acc += v[r] * G[((long)r * n + idx[k]) * r1 + s];
      w[s] = acc;
    }
    for (int s = 0; s < r1; ++s) v[s] = w[s];
  }
  reinterpret_cast<Tc*>(a.out)[e] = v[0];
}

// Workgroups of the lift: eight per compute unit.
const int kLiftGrid = 2048;

hipError_t launch_lift(ttc_dtype dt, const LiftArgs& a, int total_lines, hipStream_t s) {
  if (total_lines <= 0) return hipSuccess;
  const int grid = std::min(total_lines, kLiftGrid);
  switch (dt) {
    case TTC_F64: hipLaunchKernelGGL((lift_kernel<double, double>), dim3(grid), dim3(256), 0, s, a, total_lines); break;
    case TTC_F32: hipLaunchKernelGGL((lift_kernel<float, float>), dim3(grid), dim3(256), 0, s, a, total_lines); break;
    default: hipLaunchKernelGGL((lift_kernel<bf16_t, float>), dim3(grid), dim3(256), 0, s, a, total_lines); break;
  }
  return hipGetLastError();
}

hipError_t launch_dense(bool f64, const DenseArgs& a, hipStream_t s) {
  if (a.numel <= 0) return hipSuccess;
  const long blocks = (a.numel + 255) / 256;
  if (f64)
    hipLaunchKernelGGL((dense_kernel<double>), dim3((unsigned)blocks), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((dense_kernel<float>), dim3((unsigned)blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace ttc
