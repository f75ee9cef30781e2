// BF16 matrix product for the TT layer's dense schedule on the 16x16x32 BF16
// MFMA with FP32 accumulation:
//   C[m, n] = alpha * sum_k A[m, k] B[n, k]     (A: M x K, B: N x K, both BF16
//   with k contiguous; C: M x N FP32, row stride ldc)
// and the conversions that give it its operands: FP32 -> BF16 (round to
// nearest even) in place of layout, or transposed through LDS tiles, so that
// every product of the layer (Y = X W^T, dX = dY W, dW = dY^T X) reads both
// operands as contiguous 16-byte runs along k.
//
// Tiling: a 512-thread workgroup (8 waves, 4 x 2) computes a 256 x 256 tile,
// each wave 64 x 128 as 4 x 8 tiles of 16 x 16 (128 FP32 accumulators per
// lane).  k advances 64 at a time through two LDS buffers (each operand tile
// 256 rows x 64 k, 128-byte rows whose eight 16-byte chunks are stored in
// the order chunk ^ ((row / 2) % 8), so that the 16 lanes of a fragment read
// (16 rows, one chunk) and of a staging write (two rows, eight chunks each)
// fall on distinct banks): the next k-slice's global loads (four 16-byte
// loads per operand per thread) are issued before the current slice's MFMAs
// and stored to the other buffer after them.  Workgroups are dealt to the
// XCDs round-robin; the tile index is remapped so that each XCD walks a
// contiguous range of tiles, in groups of eight tile rows, which keeps the
// operand panels one XCD touches in its own L2.  Optional split-K writes FP32
// partial slabs that a second kernel sums in a fixed order.
#include "ttc_device.hpp"
#include "ttc_layer.h"

namespace ttc {

#define G16_BM 256
#define G16_BN 256
#define G16_BK 64
#define G16_P G16_BK
#define G16_THREADS 512

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

size_t gemm16_lds_bytes() { return (size_t)2 * 2 * G16_BM * G16_P * sizeof(uint16_t); }

namespace {

__device__ __forceinline__ void g16_load(const uint16_t* P, long ld, int row0, int nrows, int k0, int kend,
                                         u32x4* r) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int c = threadIdx.x + G16_THREADS * q;
    const int row = c >> 3, kc = (c & 7) * 8;
    u32x4 v = {0u, 0u, 0u, 0u};
    if (row0 + row < nrows && k0 + kc < kend)
      v = *reinterpret_cast<const u32x4*>(P + (long)(row0 + row) * ld + k0 + kc);
    r[q] = v;
  }
}

__device__ __forceinline__ void g16_store(uint16_t* S, const u32x4* r) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int c = threadIdx.x + G16_THREADS * q;
    const int row = c >> 3, kc = (c & 7) * 8;
    *reinterpret_cast<u32x4*>(S + row * G16_P + ((kc >> 3) ^ ((row >> 1) & 7)) * 8) = r[q];
  }
}

}  // namespace

__global__ __launch_bounds__(G16_THREADS) void gemm16_kernel(Gemm16Args g) {
  extern __shared__ __align__(16) unsigned char smem[];
  uint16_t* As = reinterpret_cast<uint16_t*>(smem);   // [2][256][72]
  uint16_t* Bs = As + 2 * G16_BM * G16_P;             // [2][256][72]
  const int tiles_m = (g.M + G16_BM - 1) / G16_BM, tiles_n = (g.N + G16_BN - 1) / G16_BN;
  int tm, tn;
  xcd_tile(blockIdx.x, tiles_m, tiles_n, g.per_xcd, &tm, &tn);
  const int m0 = tm * G16_BM, n0 = tn * G16_BN;
  const int kper = ((g.K + g.splits - 1) / g.splits + G16_BK - 1) / G16_BK * G16_BK;
  const int kbeg = blockIdx.y * kper;
  const int kend = min(g.K, kbeg + kper);
  const int nk = kend > kbeg ? (kend - kbeg + G16_BK - 1) / G16_BK : 0;

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave >> 1, wn = wave & 1;  // 4 x 2 waves: 64 rows x 128 columns each
  const int li = lane & 15, lg = lane >> 4;
  f32x4 acc[4][8];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  u32x4 ra[4], rb[4];
  if (nk > 0) {
    g16_load(g.A, g.lda, m0, g.M, kbeg, kend, ra);
    g16_load(g.B, g.ldb, n0, g.N, kbeg, kend, rb);
    g16_store(As, ra);
    g16_store(Bs, rb);
  }
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) {
      const int k0 = kbeg + (kt + 1) * G16_BK;
      g16_load(g.A, g.lda, m0, g.M, k0, kend, ra);
      g16_load(g.B, g.ldb, n0, g.N, k0, kend, rb);
    }
    // rows wm*64 + 16i + li (resp. wn*128 + 16j + li) have (row / 2) % 8 = li / 2
    const int swz = (li >> 1) & 7;
    const uint16_t* a_s = As + buf * G16_BM * G16_P + (wm * 64 + li) * G16_P;
    const uint16_t* b_s = Bs + buf * G16_BN * G16_P + (wn * 128 + li) * G16_P;
#pragma unroll
    for (int kk = 0; kk < G16_BK; kk += 32) {
      const int ch = (((kk >> 3) + lg) ^ swz) * 8;
      bf16x8 av[4], bv[8];
#pragma unroll
      for (int i = 0; i < 4; ++i) av[i] = *reinterpret_cast<const bf16x8*>(a_s + 16 * i * G16_P + ch);
#pragma unroll
      for (int j = 0; j < 8; ++j) bv[j] = *reinterpret_cast<const bf16x8*>(b_s + 16 * j * G16_P + ch);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
    if (kt + 1 < nk) {
      g16_store(As + (buf ^ 1) * G16_BM * G16_P, ra);
      g16_store(Bs + (buf ^ 1) * G16_BN * G16_P, rb);
    }
    __syncthreads();
  }
  float* C = g.splits > 1 ? g.slab + (long)blockIdx.y * g.M * g.N : g.C;
  const long ldc = g.splits > 1 ? g.N : g.ldc;
  const float alpha = g.splits > 1 ? 1.f : g.alpha;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int m = m0 + wm * 64 + 16 * i + 4 * lg + v;
      if (m >= g.M) continue;
      float* crow = C + (long)m * ldc;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int n = n0 + wn * 128 + 16 * j + li;
        if (n < g.N) crow[n] = alpha * acc[i][j][v];
      }
    }
}

// dst[e] = bf16(src[e]) for n elements (8 per thread; n a multiple of 8, both
// 16-byte aligned).
__global__ __launch_bounds__(256) void cvt16_kernel(const float* __restrict__ src, uint16_t* __restrict__ dst, long n8) {
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n8; e += (long)gridDim.x * blockDim.x) {
    const f32x4 a = reinterpret_cast<const f32x4*>(src)[2 * e];
    const f32x4 b = reinterpret_cast<const f32x4*>(src)[2 * e + 1];
    u32x4 w;
    w[0] = (uint32_t)f32_to_bf16(a[0]) | ((uint32_t)f32_to_bf16(a[1]) << 16);
    w[1] = (uint32_t)f32_to_bf16(a[2]) | ((uint32_t)f32_to_bf16(a[3]) << 16);
    w[2] = (uint32_t)f32_to_bf16(b[0]) | ((uint32_t)f32_to_bf16(b[1]) << 16);
    w[3] = (uint32_t)f32_to_bf16(b[2]) | ((uint32_t)f32_to_bf16(b[3]) << 16);
    reinterpret_cast<u32x4*>(dst)[e] = w;
  }
}

// dst[c * rows + r] = bf16(src[r * cols + c]) (and, BOTH, dst[r * cols + c]
// = bf16(src[r * cols + c])): 64 x 64 tiles through LDS (pitch 65: the
// column reads are conflict-free), the source read as 16-byte runs of a
// row, the transposed copy written as 16-byte runs (eight elements) of a
// destination row.  VEC: cols a multiple of 4 and rows of 8 (and aligned
// buffers), else one element per access.
template <bool BOTH, bool VEC>
__global__ __launch_bounds__(256) void cvt16_tr_kernel(const float* __restrict__ src, uint16_t* __restrict__ dst,
                                                       uint16_t* __restrict__ dst_t, long rows, long cols) {
  __shared__ float tile[64][65];
  const long r0 = (long)blockIdx.x * 64, c0 = (long)blockIdx.y * 64;
  if (VEC) {
    // 16 lanes per source row (four columns each), 16 rows per pass
    const int tc = (threadIdx.x & 15) * 4, tr = threadIdx.x >> 4;
#pragma unroll
    for (int q = 0; q < 64; q += 16) {
      const long r = r0 + tr + q, c = c0 + tc;
      f32x4 v = {0.f, 0.f, 0.f, 0.f};
      if (r < rows && c < cols) {
        v = *reinterpret_cast<const f32x4*>(src + r * cols + c);
        if (BOTH) {
          uint2 w;
          w.x = (uint32_t)f32_to_bf16(v[0]) | ((uint32_t)f32_to_bf16(v[1]) << 16);
          w.y = (uint32_t)f32_to_bf16(v[2]) | ((uint32_t)f32_to_bf16(v[3]) << 16);
          *reinterpret_cast<uint2*>(dst + r * cols + c) = w;
        }
      }
#pragma unroll
      for (int x = 0; x < 4; ++x) tile[tr + q][tc + x] = v[x];
    }
    __syncthreads();
    // 8 lanes per destination row (eight source rows each), 32 rows per pass
    const int dr = (threadIdx.x & 7) * 8, dc = threadIdx.x >> 3;
#pragma unroll
    for (int q = 0; q < 64; q += 32) {
      const long c = c0 + dc + q, r = r0 + dr;
      if (c < cols && r < rows) {
        u32x4 w;
#pragma unroll
        for (int x = 0; x < 4; ++x)
          w[x] = (uint32_t)f32_to_bf16(tile[dr + 2 * x][dc + q]) |
                 ((uint32_t)f32_to_bf16(tile[dr + 2 * x + 1][dc + q]) << 16);
        *reinterpret_cast<u32x4*>(dst_t + c * rows + r) = w;
      }
    }
  } else {
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;  // 64 x 4
#pragma unroll 4
    for (int q = 0; q < 64; q += 4) {
      const long r = r0 + ty + q, c = c0 + tx;
      const bool in = r < rows && c < cols;
      const float v = in ? src[r * cols + c] : 0.f;
      tile[ty + q][tx] = v;
      if (BOTH && in) dst[r * cols + c] = f32_to_bf16(v);
    }
    __syncthreads();
#pragma unroll 4
    for (int q = 0; q < 64; q += 4) {
      const long c = c0 + ty + q, r = r0 + tx;
      if (r < rows && c < cols) dst_t[c * rows + r] = f32_to_bf16(tile[tx][ty + q]);
    }
  }
}

template <bool BOTH>
static void launch_tr(const float* src, uint16_t* dst, uint16_t* dst_t, long rows, long cols, hipStream_t s) {
  const dim3 grid((unsigned)((rows + 63) / 64), (unsigned)((cols + 63) / 64));
  const bool vec = cols % 4 == 0 && rows % 8 == 0 && ((uintptr_t)src & 15) == 0 && ((uintptr_t)dst_t & 15) == 0 &&
                   (!BOTH || ((uintptr_t)dst & 7) == 0);
  if (vec)
    hipLaunchKernelGGL((cvt16_tr_kernel<BOTH, true>), grid, dim3(256), 0, s, src, dst, dst_t, rows, cols);
  else
    hipLaunchKernelGGL((cvt16_tr_kernel<BOTH, false>), grid, dim3(256), 0, s, src, dst, dst_t, rows, cols);
}

hipError_t launch_cvt16_both(const float* src, uint16_t* dst, uint16_t* dst_t, long rows, long cols, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  launch_tr<true>(src, dst, dst_t, rows, cols, s);
  return hipGetLastError();
}

hipError_t gemm16_set_lds() {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&gemm16_kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)gemm16_lds_bytes());
}

hipError_t launch_gemm16(const Gemm16Args& g, hipStream_t s) {
  const int tiles = ((g.M + G16_BM - 1) / G16_BM) * ((g.N + G16_BN - 1) / G16_BN);
  hipLaunchKernelGGL(gemm16_kernel, dim3(tiles, g.splits), dim3(G16_THREADS), gemm16_lds_bytes(), s, g);
  return hipGetLastError();
}

hipError_t launch_cvt16(const float* src, uint16_t* dst, long n, hipStream_t s) {
  const long n8 = n / 8;
  if (n8 <= 0) return hipSuccess;
  const int blocks = (int)std::min<long>((n8 + 255) / 256, 8192);
  hipLaunchKernelGGL(cvt16_kernel, dim3(blocks), dim3(256), 0, s, src, dst, n8);
  return hipGetLastError();
}

hipError_t launch_cvt16_t(const float* src, uint16_t* dst, long rows, long cols, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  launch_tr<false>(src, nullptr, dst, rows, cols, s);
  return hipGetLastError();
}

}  // namespace ttc
