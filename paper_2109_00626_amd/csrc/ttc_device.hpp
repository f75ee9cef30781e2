// Device-side helpers shared by the gfx950 kernels: element conversions,
// MFMA wrappers and a workgroup-level matrix product on 16x16 MFMA tiles.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ttc {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// BF16 storage: raw 16-bit pattern (upper half of an FP32).
struct bf16_t {
  uint16_t bits;
};

__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// FP32 -> BF16, round to nearest even (inputs are finite).
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  uint32_t b = __float_as_uint(f);
  b += 0x7FFFu + ((b >> 16) & 1u);
  return (uint16_t)(b >> 16);
}

// floor(x / d) for the multiplier m and shift l of a divisor d (FastDiv in
// the host interface).
__device__ __forceinline__ uint32_t fdiv(uint32_t x, uint32_t m, uint32_t l) {
  return (uint32_t)(((uint64_t)__umulhi(m, x) + x) >> l);
}

// Output tile (tm, tn) of workgroup b in a grid of tiles_m x tiles_n tiles.
// Workgroups are dealt to the eight XCDs round-robin; with per_xcd (the
// tiles per XCD, tiles a multiple of 8) the index is remapped so that each
// XCD walks a contiguous range of tiles, in groups of eight tile rows, which
// keeps the operand panels one XCD touches in its own L2.
__device__ __forceinline__ void xcd_tile(int b, int tiles_m, int tiles_n, int per_xcd, int* tm, int* tn) {
  int t = b;
  if (per_xcd) t = (b & 7) * per_xcd + (b >> 3);
  const int GM = 8;
  const int span = GM * tiles_n;
  const int first = (t / span) * GM;
  const int gsz = min(tiles_m - first, GM);
  const int l = t - (t / span) * span;
  *tm = first + l % gsz;
  *tn = l / gsz;
}

template <typename Tc, typename Ts>
struct Cvt;
template <>
struct Cvt<float, float> {
  static __device__ __forceinline__ float f(float v) { return v; }
};
template <>
struct Cvt<float, bf16_t> {
  static __device__ __forceinline__ float f(bf16_t v) { return bf16_to_f32(v.bits); }
};
template <>
struct Cvt<double, double> {
  static __device__ __forceinline__ double f(double v) { return v; }
};
template <>
struct Cvt<double, float> {
  static __device__ __forceinline__ double f(float v) { return (double)v; }
};
template <typename Tc, typename Ts>
__device__ __forceinline__ Tc cvt(Ts v) {
  return Cvt<Tc, Ts>::f(v);
}

// Store a compute-type value into an output element type.
__device__ __forceinline__ void store_as(float* p, float v) { *p = v; }
__device__ __forceinline__ void store_as(double* p, double v) { *p = v; }
__device__ __forceinline__ void store_as(bf16_t* p, float v) { p->bits = f32_to_bf16(v); }

// 16x16xK MFMA step for the compute type.  Operand layout (both types):
// lane l supplies A[m = l % 16][k = l / 16] and B[k = l / 16][n = l % 16].
// Accumulator element v of lane l is D[row(l / 16, v)][n = l % 16] with
// row = 4 * (l / 16) + v for FP32 and row = 4 * v + l / 16 for FP64
// (measured on gfx950).
template <typename Tc>
struct Mfma;
template <>
struct Mfma<float> {
  typedef f32x4 acc;
  static __device__ __forceinline__ acc step(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int g, int v) { return 4 * g + v; }
};
template <>
struct Mfma<double> {
  typedef f64x4 acc;
  static __device__ __forceinline__ acc step(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int g, int v) { return 4 * v + g; }
};

// Strided view of a family of matrices: element (m, k) of member (b, r) is
//   p[b * sb + r * sr + m * s0 + k * s1].
// b indexes independent products, r indexes products that are summed.
template <typename T>
struct MatView {
  const T* p;
  int s0, s1;   // row / column strides
  int sr, sb;   // summed-member / independent-member strides
};

template <typename T>
struct OutView {
  T* p;
  int s0, s1, sb;
};

// Workgroup matrix product on MFMA tiles:
//   C_b(m, n) = alpha * sum_{r < nred} sum_{k < K} A_{b,r}(m, k) B_{b,r}(k, n)  (+ C_b if accumulate)
// for b < nbat.  Every wave takes 16x16 output tiles round-robin over
// (b, tile), so calls with equal (M, N, nbat) give every tile to the same
// wave and accumulation across calls is race-free without a barrier.
// Out-of-range operand elements read as zero; out-of-range outputs are not
// written.  The caller synchronises before (operands ready) and after
// (results visible to other waves).
template <typename Tc, typename TA, typename TB, typename TC>
__device__ void wg_gemm(int M, int N, int K, int nbat, int nred, MatView<TA> A, MatView<TB> B,
                        OutView<TC> C, bool accumulate, Tc alpha = (Tc)1) {
  typedef typename Mfma<Tc>::acc acc_t;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  const int tm = (M + 15) >> 4, tn = (N + 15) >> 4;
  const int tiles = tm * tn;
  const int li = lane & 15, lk = lane >> 4;
  for (int t = wave; t < tiles * nbat; t += nw) {
    const int b = t / tiles;
    const int tt = t - b * tiles;
    const int m0 = (tt / tn) << 4, n0 = (tt % tn) << 4;
    const int am = m0 + li, bn = n0 + li;
    const bool am_ok = am < M, bn_ok = bn < N;
    acc_t c = {0, 0, 0, 0};
    for (int r = 0; r < nred; ++r) {
      const TA* pa = A.p + (long)b * A.sb + (long)r * A.sr + (long)(am_ok ? am : 0) * A.s0;
      const TB* pb = B.p + (long)b * B.sb + (long)r * B.sr + (long)(bn_ok ? bn : 0) * B.s1;
#pragma unroll 4
      for (int k0 = 0; k0 < K; k0 += 4) {
        const int k = k0 + lk;
        const bool kok = k < K;
        const Tc av = (am_ok && kok) ? cvt<Tc>(pa[(long)k * A.s1]) : (Tc)0;
        const Tc bv = (bn_ok && kok) ? cvt<Tc>(pb[(long)k * B.s0]) : (Tc)0;
        c = Mfma<Tc>::step(av, bv, c);
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int m = m0 + Mfma<Tc>::row(lk, v), n = n0 + li;
      if (m < M && n < N) {
        TC* q = C.p + (long)b * C.sb + (long)m * C.s0 + (long)n * C.s1;
        const Tc val = alpha * c[v];
        *q = accumulate ? (TC)(*q + val) : (TC)val;
      }
    }
  }
}

template <typename T>
__device__ __forceinline__ MatView<T> mv(const T* p, int s0, int s1, int sr = 0, int sb = 0) {
  MatView<T> v;
  v.p = p;
  v.s0 = s0;
  v.s1 = s1;
  v.sr = sr;
  v.sb = sb;
  return v;
}
template <typename T>
__device__ __forceinline__ OutView<T> ov(T* p, int s0, int s1, int sb = 0) {
  OutView<T> v;
  v.p = p;
  v.s0 = s0;
  v.s1 = s1;
  v.sb = sb;
  return v;
}

// Deterministic workgroup sum of one double per thread (blockDim <= 1024).
__device__ __forceinline__ double wg_sum_f64(double v, double* scratch) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if (lane == 0) scratch[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    for (int w = 0; w < nw; ++w) s += scratch[w];
    scratch[0] = s;
  }
  __syncthreads();
  s = scratch[0];
  __syncthreads();
  return s;
}

}  // namespace ttc
