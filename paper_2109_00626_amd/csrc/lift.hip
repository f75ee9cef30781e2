// Output forms of a shared-block contraction.
//
// Natural-order TT (eq. (8) mode order, Algorithm 2's final permutation
// realised on cores): the junction matrix K (kr x Q) is absorbed into the
// free core next to it and its column index q is carried through the other
// side's cores as an extra bond factor (merged index (own bond) * Q + q).
// The carried-bond cores are block-diagonal copies: almost all of their
// entries are zero, so the kernel is a pure HBM write stream: the cores
// are written as one stream of 16-byte runs (consecutive outputs of one row
// bond and mode index), the block-diagonal ones with at most one source
// load per run.
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

template <typename T>
struct Vec16;
template <>
struct Vec16<float> {
  typedef float type __attribute__((ext_vector_type(4)));
};
template <>
struct Vec16<double> {
  typedef double type __attribute__((ext_vector_type(2)));
};

#ifndef LIFT_UNROLL
#define LIFT_UNROLL 1
#endif
constexpr int kLiftUnroll = LIFT_UNROLL;

// The output cores as one stream of items (a run of `vec` consecutive
// outputs of one line; 16 bytes when the line length allows).  A thread
// takes kLiftUnroll items a grid stride apart and computes all of them
// (issuing their source loads together) before it stores any.  One item
// per pass is the fastest: loads and stores share one completion counter,
// so each pass's source loads also wait for the stores issued before them,
// and more items per pass only lengthen that wait (natural-form output of
// the order-10 pair, 204 MB: 34.5 us with one item, 39 with two, 44 with
// four, 83 with eight).  Item ranges start at multiples of 64, so a wave's
// items lie in one core and the core lookup is uniform.
template <typename Tin, typename Tc>
__global__ __launch_bounds__(256) void lift_kernel(LiftArgs a, long total_items) {
  constexpr int VW = 16 / sizeof(Tc);
  typedef typename Vec16<Tc>::type vec_t;
  const Tc* K = reinterpret_cast<const Tc*>(a.K);
  const long stride = (long)gridDim.x * blockDim.x;
  const int lane = threadIdx.x & 63;
  int cc[kLiftUnroll];
#pragma unroll
  for (int u = 0; u < kLiftUnroll; ++u) cc[u] = 0;
  for (long w0 = (long)blockIdx.x * blockDim.x + (threadIdx.x & ~63); w0 < total_items;
       w0 += kLiftUnroll * stride) {
    vec_t v[kLiftUnroll];
    Tc* p[kLiftUnroll];
#pragma unroll
    for (int u = 0; u < kLiftUnroll; ++u) {
      p[u] = nullptr;
      const long ew = w0 + u * stride;  // the wave's first item
      if (ew >= total_items) continue;
      int k = cc[u];
      while (k + 1 < a.ncores && a.c[k + 1].item_begin <= ew) ++k;
      k = __builtin_amdgcn_readfirstlane(k);
      cc[u] = k;
      const LiftCore& c = a.c[k];
      const long t = ew + lane - c.item_begin;
      if (t >= c.items) continue;
      long l;
      int j;
      if (c.items <= 0xffffffffL) {
        const uint32_t ll = fdiv((uint32_t)t, c.fw.m, c.fw.l);
        l = ll;
        j = ((int)((uint32_t)t - ll * (uint32_t)c.w)) * c.vec;
      } else {
        l = t / c.w;
        j = (int)(t - l * c.w) * c.vec;
      }
      const int row = (int)fdiv((uint32_t)l, c.fn.m, c.fn.l), i = (int)l - row * c.n;
      p[u] = reinterpret_cast<Tc*>(c.dst) + l * c.d1 + j;
      if (c.vec == 1) {
        v[u][0] = lift_value<Tin, Tc>(c, K, a.Q, row, i, j);
      } else if (c.op == LIFT_DELTA && a.Q % VW == 0) {
        // block-diagonal copy: line (row = ra * Q + q, i) holds entries only
        // at the columns b * Q + q, so this run holds at most one (at slot
        // s) and needs at most one load
        const int ra = (int)fdiv((uint32_t)row, a.fq.m, a.fq.l), q = row - ra * a.Q;
        const int b = (int)fdiv((uint32_t)j, a.fq.m, a.fq.l), sl = q - (j - b * a.Q);
        Tc e = (Tc)0;
        if (sl >= 0 && sl < VW) e = cvt<Tc>(reinterpret_cast<const Tin*>(c.src)[((long)ra * c.n + i) * c.r1 + b]);
#pragma unroll
        for (int x = 0; x < VW; ++x) v[u][x] = x == sl ? e : (Tc)0;
      } else {
#pragma unroll
        for (int x = 0; x < VW; ++x) v[u][x] = lift_value<Tin, Tc>(c, K, a.Q, row, i, j + x);
      }
    }
#pragma unroll
    for (int u = 0; u < kLiftUnroll; ++u) {
      if (!p[u]) continue;
      if (a.c[cc[u]].vec == 1)
        *p[u] = v[u][0];
      else
        __builtin_nontemporal_store(v[u], reinterpret_cast<vec_t*>(p[u]));
    }
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

// Workgroups of the lift at most (a grid-stride loop covers the rest).
#ifndef LIFT_GRID
#define LIFT_GRID 8192
#endif
const long kLiftGrid = LIFT_GRID;

hipError_t launch_lift(ttc_dtype dt, const LiftArgs& in, int total_lines, hipStream_t s) {
  if (total_lines <= 0) return hipSuccess;
  LiftArgs a = in;
  const int VW = dt == TTC_F64 ? 2 : 4;
  a.fq = make_fastdiv((uint32_t)std::max(a.Q, 1));
  long items = 0;
  for (int k = 0; k < a.ncores; ++k) {
    LiftCore& c = a.c[k];
    const bool v = c.d1 % VW == 0 && ((uintptr_t)c.dst & 15) == 0;
    c.vec = v ? VW : 1;
    c.w = c.d1 / c.vec;
    c.items = (long)c.d0 * c.n * c.w;
    c.item_begin = items;
    c.fw = make_fastdiv((uint32_t)std::max(c.w, 1));
    c.fn = make_fastdiv((uint32_t)std::max(c.n, 1));
    items += (c.items + 63) / 64 * 64;
  }
  if (items <= 0) return hipSuccess;
  const int grid = (int)std::min((items + 256L * kLiftUnroll - 1) / (256L * kLiftUnroll), kLiftGrid);
  switch (dt) {
    case TTC_F64: hipLaunchKernelGGL((lift_kernel<double, double>), dim3(grid), dim3(256), 0, s, a, items); break;
    case TTC_F32: hipLaunchKernelGGL((lift_kernel<float, float>), dim3(grid), dim3(256), 0, s, a, items); break;
    default: hipLaunchKernelGGL((lift_kernel<bf16_t, float>), dim3(grid), dim3(256), 0, s, a, items); break;
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
