// TT-matrix times a dense batch (a TT layer), its backward, and the MSE loss.
//
// Dense schedule: the TT-matrix is rebuilt from its cores by a chain of
// matrix products L_{k+1} = L_k . W^(k) (W^(k) viewed as R_k x (I_k J_k R_{k+1})),
// whose result indexes the pair modes m_k = (i_k, j_k) with m_0 slowest; a
// permutation then gives W[i, j] with little-endian row and column indices.
// The batch product is one MFMA GEMM.  The backward forms dW = dY^T X,
// permutes it back to pair-mode order and projects it onto each core:
//   dG^(k)[r, m_k, s] = sum_{m_<k} L_k[m_<k, r] Rt_k[m_<k, m_k, s],
// with the right environments Rt_{k-1} = Rt_k . W^(k)^T (Rt_{N-1} = dW).
// Every contraction is the GEMM kernel below.
//
// Core-by-core schedule (the method applied to the batch): with X viewed as
// Z_0[P_0, Q_0, J_0, R_0] (P_k = (b, j_{d-1}..j_{k+1}), Q_k = (i_{k-1}..i_0),
// i_0 fastest), step k contracts (j_k, r_k) with the core:
//   Z_{k+1}[(P_k, Q_k), (i_k, r_{k+1})] = Z_k[(P_k, Q_k), (j_k, r_k)] . Wp_k
// with Wp_k[(j, r), (i, r1)] = G^(k)[r, i, j, r1].  The GEMM's store writes
// each result straight into the layout the next step reads,
// [P_{k+1}, (i_k, Q_k), j_{k+1}, r_{k+1}], and the last step into
// Y[b, i_{d-1}..i_0].  The backward gathers each step's output gradient
// through the same map, then dZ_k = dC_k Wp_k^T and dWp_k = Z_k^T dC_k.
//
// GEMM: 128 x 128 output tile per 256-thread workgroup, each wave a 64 x 64
// quarter on MFMA tiles (FP32: 32x32x2, BF16: 16x16x32 with FP32
// accumulation), operands staged through double-buffered LDS; thin tiles
// (32 x 128, 128 x 32, 128 x 64; FP32 on 16x16x4) for the rank-sized
// products of the core chain, so that a side of 32 is not padded to 128.  Global
// operands are FP32; the BF16 variant rounds them (RNE) while staging.
// Optional split-K writes FP32 partial slabs that a second kernel sums in a
// fixed order (deterministic).
#include "ttc_device.hpp"
#include "ttc_layer.h"

namespace ttc {

#define GPAD 4

template <bool BF16>
struct GemmCfg;
// FP32: K slices of 16 (three workgroups' double-buffered tiles fit one
// CU's LDS) with registers bounded for three waves per SIMD (the FP32
// kernels' spills are in the epilogue only); BF16: K slices of 64, no
// register bound.  On the 8192 x 4096 x 4096 forward product this runs at
// 120 TFLOP/s against 117 with K slices of 32 and two waves per SIMD.
#ifndef GEMM_F32_BK
#define GEMM_F32_BK 16
#endif
template <>
struct GemmCfg<false> {
  static constexpr int BK = GEMM_F32_BK;
};
template <>
struct GemmCfg<true> {
  static constexpr int BK = 64;
};

// Output tile shapes (TM x TN per 256-thread workgroup): the square tile
// and thin ones for products with a side of 32 or 64 (rank-sized), each
// wave computing a (TM / WM) x (TN / WN) block of FI x FJ MFMA tiles.
template <int TM, int TN>
struct GemmShape {
  static constexpr int WN = (TM == 128 && TN == 32) ? 1 : (TM == 32 ? 4 : 2);
  static constexpr int WM = 4 / WN;
  static constexpr int FI = TM / WM / 16, FJ = TN / WN / 16;
};

// Number of float4 loads per thread for one operand tile of ROWS rows.
template <bool BF16, int ROWS>
__device__ constexpr int loads_per_thread() {
  return (ROWS * GemmCfg<BF16>::BK / 4 + 255) / 256;
}

// Load one operand tile (rows = the operand's M or N dimension, ROWS of
// them; columns = 32/64 of K) into registers.  kc: K is the contiguous
// dimension.
template <bool BF16, bool KC, int ROWS>
__device__ __forceinline__ void load_tile(const float* P, long ld, int row0, int nrows, int k0, int K, bool vec,
                                          f32x4* r) {
  constexpr int BK = GemmCfg<BF16>::BK;
  constexpr int L = loads_per_thread<BF16, ROWS>();
#pragma unroll
  for (int it = 0; it < L; ++it) {
    const int e = threadIdx.x + 256 * it;
    int row, kk;
    if (KC) {
      row = e / (BK / 4);
      kk = (e % (BK / 4)) * 4;
    } else {
      kk = e / (ROWS / 4);
      row = (e % (ROWS / 4)) * 4;
    }
    f32x4 v = {0.f, 0.f, 0.f, 0.f};
    if ((ROWS * BK / 4) % 256 != 0 && e >= ROWS * BK / 4) {
    } else if (KC) {
      const int gr = row0 + row, gk = k0 + kk;
      if (gr < nrows) {
        const float* p = P + (long)gr * ld + gk;
        if (vec && gk + 3 < K) {
          v = *reinterpret_cast<const f32x4*>(p);
        } else {
#pragma unroll
          for (int q = 0; q < 4; ++q)
            if (gk + q < K) v[q] = p[q];
        }
      }
    } else {
      const int gr = row0 + row, gk = k0 + kk;
      if (gk < K) {
        const float* p = P + (long)gk * ld + gr;
        if (vec && gr + 3 < nrows) {
          v = *reinterpret_cast<const f32x4*>(p);
        } else {
#pragma unroll
          for (int q = 0; q < 4; ++q)
            if (gr + q < nrows) v[q] = p[q];
        }
      }
    }
    r[it] = v;
  }
}

// Store staged registers into LDS.  FP32 layout: S[k][row] (pitch
// ROWS+GPAD); BF16 layout: S[row][k] (pitch BK+8, k contiguous for 16-byte
// fragments).
template <bool BF16, bool KC, int ROWS>
__device__ __forceinline__ void store_tile(void* S, const f32x4* r) {
  constexpr int BK = GemmCfg<BF16>::BK;
  constexpr int L = loads_per_thread<BF16, ROWS>();
#pragma unroll
  for (int it = 0; it < L; ++it) {
    const int e = threadIdx.x + 256 * it;
    int row, kk;
    if (KC) {
      row = e / (BK / 4);
      kk = (e % (BK / 4)) * 4;
    } else {
      kk = e / (ROWS / 4);
      row = (e % (ROWS / 4)) * 4;
    }
    if ((ROWS * BK / 4) % 256 != 0 && e >= ROWS * BK / 4) continue;
    if (!BF16) {
      float* s = reinterpret_cast<float*>(S);
      if (KC) {
#pragma unroll
        for (int q = 0; q < 4; ++q) s[(kk + q) * (ROWS + GPAD) + row] = r[it][q];
      } else {
        *reinterpret_cast<f32x4*>(s + kk * (ROWS + GPAD) + row) = r[it];
      }
    } else {
      uint16_t* s = reinterpret_cast<uint16_t*>(S);
      constexpr int P = BK + 8;
      if (KC) {
        uint2 w;
        w.x = (uint32_t)f32_to_bf16(r[it][0]) | ((uint32_t)f32_to_bf16(r[it][1]) << 16);
        w.y = (uint32_t)f32_to_bf16(r[it][2]) | ((uint32_t)f32_to_bf16(r[it][3]) << 16);
        *reinterpret_cast<uint2*>(s + row * P + kk) = w;
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) s[(row + q) * P + kk] = f32_to_bf16(r[it][q]);
      }
    }
  }
}

template <bool BF16, int ROWS>
__host__ __device__ constexpr int tile_elems() {
  return BF16 ? ROWS * (GemmCfg<true>::BK + 8) : GemmCfg<false>::BK * (ROWS + GPAD);
}

#ifndef GEMM_WPE
#define GEMM_WPE 3
#endif
// W32 (FP32 128 x 128 tiles with a plain or batched store and no K
// split): the 32x32x2 MFMA in place of 16x16x4.
template <bool A_KC, bool B_KC, bool BF16, int TM, int TN, bool W32 = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(BF16 ? 1 : GEMM_WPE))) void gemm_kernel(GemmArgs g) {
  extern __shared__ __align__(16) unsigned char smem[];
  typedef GemmShape<TM, TN> S;
  constexpr int FI = S::FI, FJ = S::FJ;
  constexpr int BK = GemmCfg<BF16>::BK;
  constexpr int LA = loads_per_thread<BF16, TM>(), LB = loads_per_thread<BF16, TN>();
  constexpr int esz = BF16 ? 2 : 4;
  constexpr int TA = tile_elems<BF16, TM>(), TB = tile_elems<BF16, TN>();
  unsigned char* As = smem;                    // [2][TA]
  unsigned char* Bs = smem + 2 * TA * esz;     // [2][TB]
  const int tn = (g.N + TN - 1) / TN;
  const int bm = blockIdx.x / tn, bn = blockIdx.x - bm * tn;
  const int m0 = bm * TM, n0 = bn * TN;
  // K range of this split
  const int kper = ((g.K + g.splits - 1) / g.splits + BK - 1) / BK * BK;
  const int kbeg = blockIdx.y * kper;
  const int kend = min(g.K, kbeg + kper);
  const int nk = kend > kbeg ? (kend - kbeg + BK - 1) / BK : 0;
  const float* const Ag = g.A + (long)blockIdx.z * g.sa;  // batch member (z = 0 unless batched)
  const float* const Bg = g.B + (long)blockIdx.z * g.sb;

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave / S::WN, wn = wave % S::WN;
  const int li = lane & 15, lg = lane >> 4;
  const int am = wm * FI * 16, bn0 = wn * FJ * 16;  // the wave's block
  f32x4 acc[FI][FJ];
#pragma unroll
  for (int i = 0; i < FI; ++i)
#pragma unroll
    for (int j = 0; j < FJ; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  // each wave's 64 x 64 block as 2 x 2 tiles of the 32x32x2 MFMA (half the
  // MFMA instructions of 16x16x4 tiles, and the epilogue's columns 32 lanes
  // wide): forward + backward of the order-4 layer 7.05-7.13 ms against
  // 7.22-7.24 with 16x16x4 tiles.  The relayout-store and split-K products
  // of the core-by-core schedule keep 16x16x4 (with 32x32x2 there, 38.7-39.0
  // ms against 38.2 for its forward + backward; its split-K core gradients
  // took 5.2 ms against 4.8)
  constexpr bool M32 = W32 && !BF16 && TM == 128 && TN == 128;
  typedef float f32x16 __attribute__((ext_vector_type(16)));
  f32x16 acc32[2][2];
  if constexpr (M32) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc32[i][j][r] = 0.f;
  }

  f32x4 ra[LA], rb[LB];
  if (nk > 0) {
    load_tile<BF16, A_KC, TM>(Ag, g.lda, m0, g.M, kbeg, kend, g.vec_a, ra);
    load_tile<BF16, B_KC, TN>(Bg, g.ldb, n0, g.N, kbeg, kend, g.vec_b, rb);
    store_tile<BF16, A_KC, TM>(As, ra);
    store_tile<BF16, B_KC, TN>(Bs, rb);
  }
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) {
      const int k0 = kbeg + (kt + 1) * BK;
      load_tile<BF16, A_KC, TM>(Ag, g.lda, m0, g.M, k0, kend, g.vec_a, ra);
      load_tile<BF16, B_KC, TN>(Bg, g.ldb, n0, g.N, k0, kend, g.vec_b, rb);
    }
    if constexpr (M32) {
      // 32x32x2 MFMA: lane l supplies A[m = l % 32][k = l / 32] and
      // B[k = l / 32][n = l % 32]
      const float* a_s = reinterpret_cast<const float*>(As) + buf * TA;
      const float* b_s = reinterpret_cast<const float*>(Bs) + buf * TB;
      const int l32 = lane & 31, h = lane >> 5;
#pragma unroll
      for (int kk = 0; kk < BK; kk += 2) {
        float av[2], bv[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) av[i] = a_s[(kk + h) * (TM + GPAD) + am + 32 * i + l32];
#pragma unroll
        for (int j = 0; j < 2; ++j) bv[j] = b_s[(kk + h) * (TN + GPAD) + bn0 + 32 * j + l32];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j)
            acc32[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[i], bv[j], acc32[i][j], 0, 0, 0);
      }
    } else if (!BF16) {
      const float* a_s = reinterpret_cast<const float*>(As) + buf * TA;
      const float* b_s = reinterpret_cast<const float*>(Bs) + buf * TB;
#pragma unroll
      for (int kk = 0; kk < BK; kk += 4) {
        float av[FI], bv[FJ];
#pragma unroll
        for (int i = 0; i < FI; ++i) av[i] = a_s[(kk + lg) * (TM + GPAD) + am + 16 * i + li];
#pragma unroll
        for (int j = 0; j < FJ; ++j) bv[j] = b_s[(kk + lg) * (TN + GPAD) + bn0 + 16 * j + li];
#pragma unroll
        for (int i = 0; i < FI; ++i)
#pragma unroll
          for (int j = 0; j < FJ; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i], bv[j], acc[i][j], 0, 0, 0);
      }
    } else {
      const uint16_t* a_s = reinterpret_cast<const uint16_t*>(As) + buf * TA;
      const uint16_t* b_s = reinterpret_cast<const uint16_t*>(Bs) + buf * TB;
      constexpr int P = BK + 8;
#pragma unroll
      for (int kk = 0; kk < BK; kk += 32) {
        bf16x8 av[FI], bv[FJ];
#pragma unroll
        for (int i = 0; i < FI; ++i)
          av[i] = *reinterpret_cast<const bf16x8*>(a_s + (am + 16 * i + li) * P + kk + 8 * lg);
#pragma unroll
        for (int j = 0; j < FJ; ++j)
          bv[j] = *reinterpret_cast<const bf16x8*>(b_s + (bn0 + 16 * j + li) * P + kk + 8 * lg);
#pragma unroll
        for (int i = 0; i < FI; ++i)
#pragma unroll
          for (int j = 0; j < FJ; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[i], bv[j], acc[i][j], 0, 0, 0);
      }
    }
    if (kt + 1 < nk) {
      store_tile<BF16, A_KC, TM>(As + (buf ^ 1) * TA * esz, ra);
      store_tile<BF16, B_KC, TN>(Bs + (buf ^ 1) * TB * esz, rb);
    }
    __syncthreads();
  }
  float* C = g.splits > 1 ? g.slab + (long)blockIdx.y * g.M * g.N : g.C + (long)blockIdx.z * g.sc;
  const long ldc = g.splits > 1 ? g.N : g.ldc;
  const float alpha = g.splits > 1 ? 1.f : g.alpha;
  if constexpr (M32) {
    // element r of a 32 x 32 accumulator: row 8 (r / 4) + 4 (l / 32) + r % 4,
    // column l % 32
    const int l32 = lane & 31, h = lane >> 5;
    if (g.mapped) {
      // relayout store: the column parts once, each row part once (32-bit
      // divisions: m, n and the radices are ints)
      long coff[2];
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int n = n0 + bn0 + 32 * j + l32;
        coff[j] = (long)(n / g.map.nr0) * g.map.ns1 + (long)(n % g.map.nr0) * g.map.ns0;
      }
      float* const Cz = g.C + (long)blockIdx.z * g.sc;
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int m = m0 + am + 32 * i + 8 * (r >> 2) + 4 * h + (r & 3);
          if (m >= g.M) continue;
          const int q = m % g.map.mr0, t = m / g.map.mr0;
          const long ro = (long)(t / g.map.mr1) * g.map.ms2 + (long)(t % g.map.mr1) * g.map.ms1 + (long)q * g.map.ms0;
#pragma unroll
          for (int j = 0; j < 2; ++j)
            if (n0 + bn0 + 32 * j + l32 < g.N) Cz[ro + coff[j]] = g.alpha * acc32[i][j][r];
        }
      return;
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int m = m0 + am + 32 * i + 8 * (r >> 2) + 4 * h + (r & 3);
          const int n = n0 + bn0 + 32 * j + l32;
          if (m < g.M && n < g.N) C[(long)m * ldc + n] = alpha * acc32[i][j][r];
        }
    return;
  }
  if (g.mapped) {
    // relayout store: row and column parts of each address computed once
    long roff[FI][4], coff[FJ];
#pragma unroll
    for (int i = 0; i < FI; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const long m = m0 + am + 16 * i + 4 * lg + v;
        const long q = m % g.map.mr0, t = m / g.map.mr0;
        roff[i][v] = (t / g.map.mr1) * g.map.ms2 + (t % g.map.mr1) * g.map.ms1 + q * g.map.ms0;
      }
#pragma unroll
    for (int j = 0; j < FJ; ++j) {
      const long n = n0 + bn0 + 16 * j + li;
      coff[j] = (n / g.map.nr0) * g.map.ns1 + (n % g.map.nr0) * g.map.ns0;
    }
#pragma unroll
    for (int i = 0; i < FI; ++i)
#pragma unroll
      for (int j = 0; j < FJ; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int m = m0 + am + 16 * i + 4 * lg + v;
          const int n = n0 + bn0 + 16 * j + li;
          if (m < g.M && n < g.N) g.C[(long)blockIdx.z * g.sc + roff[i][v] + coff[j]] = g.alpha * acc[i][j][v];
        }
    return;
  }
#pragma unroll
  for (int i = 0; i < FI; ++i)
#pragma unroll
    for (int j = 0; j < FJ; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = m0 + am + 16 * i + 4 * lg + v;
        const int n = n0 + bn0 + 16 * j + li;
        if (m < g.M && n < g.N) C[(long)m * ldc + n] = alpha * acc[i][j][v];
      }
}

// C = alpha * (sum over z of slab[z]): 256 / ZL consecutive elements per
// workgroup, ZL lanes per element, each lane summing every ZL-th partial in
// order, then the ZL sums added in lane order (a fixed order:
// deterministic).  ZL = 8, or 64 for many partials of a small output.
template <int ZL>
__global__ __launch_bounds__(256) void splitk_reduce_kernel(const float* slab, int splits, int M, int N, float alpha,
                                                            float* C, long ldc) {
  constexpr int EL = 256 / ZL;
  __shared__ float part[ZL][EL + 1];
  const int el = threadIdx.x % EL, zl = threadIdx.x / EL;
  const long MN = (long)M * N;
  const long e = (long)blockIdx.x * EL + el;
  float s = 0.f;
  if (e < MN)
    for (int z = zl; z < splits; z += ZL) s += slab[(long)z * MN + e];
  part[zl][el] = s;
  __syncthreads();
  if (zl == 0 && e < MN) {
    float t = part[0][el];
#pragma unroll
    for (int q = 1; q < ZL; ++q) t += part[q][el];
    const long m = e / N, n = e - m * N;
    C[m * ldc + n] = alpha * t;
  }
}

// Pair-mode order (m_0 slowest, m_k = i_k * J_k + j_k) <-> W[i, j] with
// little-endian i and j.  dir 0: pair -> matrix, dir 1: matrix -> pair.
// One thread per element of the destination.
__global__ __launch_bounds__(256) void permute_kernel(PermArgs p) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= p.total) return;
  long src;
  if (p.dir == 0) {
    // destination: matrix element (row, col)
    long row = e / p.cols, col = e - row * p.cols;
    long off = 0;
    for (int k = 0; k < p.d; ++k) {
      const int ik = (int)(row % p.I[k]);
      row /= p.I[k];
      const int jk = (int)(col % p.J[k]);
      col /= p.J[k];
      off += (long)(ik * p.J[k] + jk) * p.pstride[k];
    }
    src = off;
  } else {
    // destination: pair-mode element e
    long rem = e, row = 0, col = 0;
    long rs = 1, cs = 1;
    // digits from the fastest pair mode (k = d-1) to the slowest
    long ris[TTC_MAX_ORDER], cjs[TTC_MAX_ORDER];
    for (int k = p.d - 1; k >= 0; --k) {
      const int mk = (int)(rem % (p.I[k] * p.J[k]));
      rem /= (p.I[k] * p.J[k]);
      ris[k] = mk / p.J[k];
      cjs[k] = mk - ris[k] * p.J[k];
    }
    for (int k = 0; k < p.d; ++k) {
      row += ris[k] * rs;
      rs *= p.I[k];
      col += cjs[k] * cs;
      cs *= p.J[k];
    }
    src = row * p.cols + col;
  }
  p.dst[e] = p.src[src];
}

// Tiled form of the same permutation (see TilePermArgs): the tile is read
// with the source layout's contiguous digits fastest, transposed through
// LDS (pitch Bp + 1: conflict-free both ways) and written with the
// destination layout's contiguous digits fastest; V = 4: each thread moves
// four consecutive elements of a run with one 16-byte global access (8
// bytes for a BF16 destination).
template <int V, bool OUT16>
__global__ __launch_bounds__(256) void tile_permute_kernel(TilePermArgs p) {
  __shared__ float tile[kTilePermElems + 64];
  __shared__ long offP[256];
  const int Bp = p.Bp, Bm = p.Bm, pitch = Bp + 1;
  const int gp = Bp / V, gm = Bm / V, ng = Bp * Bm / V;
  // tile base offsets from the outer digits
  long rem = blockIdx.x, baseP = 0, baseM = 0;
  for (int q = 0; q < p.nout; ++q) {
    const long dq = rem % p.orad[q];
    rem /= p.orad[q];
    baseP += dq * p.osP[q];
    baseM += dq * p.osM[q];
  }
  // pair-mode offset of each combination c of the leading column digits
  for (int c = threadIdx.x; c < Bm; c += 256) {
    long r = c, o = 0;
    for (int k = 0; k < p.t; ++k) {
      o += (r % p.jrad[k]) * p.sPj[k];
      r /= p.jrad[k];
    }
    offP[c] = o;
  }
  __syncthreads();
  if (p.dir == 0) {
    // pair-mode -> matrix: read runs of Bp, write runs of Bm
    for (int g = threadIdx.x; g < ng; g += 256) {
      const int c = (int)fdiv((uint32_t)g, p.fgp.m, p.fgp.l), q = (g - c * gp) * V;
      const float* src = p.src + baseP + offP[c] + q;
      if (V == 4) {
        const f32x4 v = *reinterpret_cast<const f32x4*>(src);
#pragma unroll
        for (int x = 0; x < V; ++x) tile[c * pitch + q + x] = v[x];
      } else {
        tile[c * pitch + q] = *src;
      }
    }
    __syncthreads();
    for (int g = threadIdx.x; g < ng; g += 256) {
      const int q = (int)fdiv((uint32_t)g, p.fgm.m, p.fgm.l), c = (g - q * gm) * V;
      const int il = (int)fdiv((uint32_t)q, p.fjl.m, p.fjl.l), jl = q - il * p.Jl;
      const long o = baseM + c + il * p.sMi + jl * p.sMj;
      float v[V];
#pragma unroll
      for (int x = 0; x < V; ++x) v[x] = tile[(c + x) * pitch + q];
      if (OUT16) {
        if (V == 4) {
          uint2 w;
          w.x = (uint32_t)f32_to_bf16(v[0]) | ((uint32_t)f32_to_bf16(v[1]) << 16);
          w.y = (uint32_t)f32_to_bf16(v[2]) | ((uint32_t)f32_to_bf16(v[3]) << 16);
          *reinterpret_cast<uint2*>(p.dst16 + o) = w;
        } else {
          p.dst16[o] = f32_to_bf16(v[0]);
        }
      } else if (V == 4) {
        *reinterpret_cast<f32x4*>(p.dst + o) = f32x4{v[0], v[1], v[2], v[3]};
      } else {
        p.dst[o] = v[0];
      }
    }
  } else {
    // matrix -> pair-mode: read runs of Bm, write runs of Bp
    for (int g = threadIdx.x; g < ng; g += 256) {
      const int q = (int)fdiv((uint32_t)g, p.fgm.m, p.fgm.l), c = (g - q * gm) * V;
      const int il = (int)fdiv((uint32_t)q, p.fjl.m, p.fjl.l), jl = q - il * p.Jl;
      const float* src = p.src + baseM + c + il * p.sMi + jl * p.sMj;
      if (V == 4) {
        const f32x4 v = *reinterpret_cast<const f32x4*>(src);
#pragma unroll
        for (int x = 0; x < V; ++x) tile[(c + x) * pitch + q] = v[x];
      } else {
        tile[c * pitch + q] = *src;
      }
    }
    __syncthreads();
    for (int g = threadIdx.x; g < ng; g += 256) {
      const int c = (int)fdiv((uint32_t)g, p.fgp.m, p.fgp.l), q = (g - c * gp) * V;
      float* dst = p.dst + baseP + offP[c] + q;
      if (V == 4) {
        *reinterpret_cast<f32x4*>(dst) =
            f32x4{tile[c * pitch + q], tile[c * pitch + q + 1], tile[c * pitch + q + 2], tile[c * pitch + q + 3]};
      } else {
        *dst = tile[c * pitch + q];
      }
    }
  }
}

// dst[m * N + n] = src[map(m, n)]: one wave per destination row (rows
// grid-stride), the row's part of the map computed once per row in scalar
// registers; along the row the map is n -> (n / nr0) ns1 + (n % nr0) ns0,
// runs of nr0 consecutive elements when ns0 = 1.  vec: ns0 = 1, nr0, N and
// every row offset multiples of 4 (four elements per lane, 16-byte loads and
// stores).
__global__ __launch_bounds__(256) void gather_mapped_kernel(GatherArgs a, int vec) {
  const int lane = threadIdx.x & 63;
  const long waves = (long)gridDim.x * 4;
  const int nr0 = a.map.nr0, N = (int)a.N;
  for (long m = (long)blockIdx.x * 4 + (threadIdx.x >> 6); m < a.M; m += waves) {
    const long q = m % a.map.mr0, t = m / a.map.mr0;
    const long base = (t / a.map.mr1) * a.map.ms2 + (t % a.map.mr1) * a.map.ms1 + q * a.map.ms0;
    float* drow = a.dst + m * a.N;
    if (vec) {
      for (int n = 4 * lane; n < N; n += 256) {
        const int hi = n / nr0;
        const f32x4 v = *reinterpret_cast<const f32x4*>(a.src + base + (long)hi * a.map.ns1 + (n - hi * nr0));
        *reinterpret_cast<f32x4*>(drow + n) = v;
      }
    } else {
      for (int n = lane; n < N; n += 64) {
        const int hi = n / nr0;
        drow[n] = a.src[base + (long)hi * a.map.ns1 + (long)(n - hi * nr0) * a.map.ns0];
      }
    }
  }
}

// Core G[r, i, j, r1] (R x I x J x R1) <-> Wp[(j, r), (i, r1)], one thread
// per element of the destination.
__global__ __launch_bounds__(256) void core_perm_kernel(const float* src, float* dst, int R, int I, int J, int R1,
                                                        int dir) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long total = (long)R * I * J * R1;
  if (e >= total) return;
  if (dir == 0) {
    // e indexes Wp: ((j * R + r) * I + i) * R1 + r1
    long t = e;
    const int r1 = (int)(t % R1);
    t /= R1;
    const int i = (int)(t % I);
    t /= I;
    const int r = (int)(t % R);
    const int j = (int)(t / R);
    dst[e] = src[(((long)r * I + i) * J + j) * R1 + r1];
  } else {
    // e indexes the core: ((r * I + i) * J + j) * R1 + r1
    long t = e;
    const int r1 = (int)(t % R1);
    t /= R1;
    const int j = (int)(t % J);
    t /= J;
    const int i = (int)(t % I);
    const int r = (int)(t / I);
    dst[e] = src[(((long)j * R + r) * I + i) * R1 + r1];
  }
}

// Partial sums of (y - t)^2 per block and dy = scale * (y - t); the
// difference, its square and the sum are FP64.
__global__ __launch_bounds__(256) void mse_partial_kernel(const float* y, const float* t, long n, float* dy,
                                                          double dscale, double* partials) {
  __shared__ double scratch[16];
  double s = 0.0;
  const long stride = (long)gridDim.x * blockDim.x;
  const long n4 = n / 4;
  const f32x4* y4 = reinterpret_cast<const f32x4*>(y);
  const f32x4* t4 = reinterpret_cast<const f32x4*>(t);
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n4; e += stride) {
    const f32x4 a = y4[e], b = t4[e];
    f32x4 g;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double d = (double)a[q] - (double)b[q];
      s += d * d;
      g[q] = (float)(dscale * d);
    }
    if (dy) reinterpret_cast<f32x4*>(dy)[e] = g;
  }
  for (long e = 4 * n4 + (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
    const double d = (double)y[e] - (double)t[e];
    s += d * d;
    if (dy) dy[e] = (float)(dscale * d);
  }
  s = wg_sum_f64(s, scratch);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void mse_final_kernel(const double* partials, int nb, double inv_n, double* out) {
  __shared__ double scratch[16];
  double s = 0.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) s += partials[b];
  s = wg_sum_f64(s, scratch);
  if (threadIdx.x == 0) out[0] = s * inv_n;
}

// ------------------------------------------------------------------ launchers
template <bool A_KC, bool B_KC, bool BF16, int TM, int TN, bool W32 = false>
static hipError_t gemm_launch(const GemmArgs& g, hipStream_t s) {
  constexpr int esz = BF16 ? 2 : 4;
  const size_t lds = (size_t)2 * (tile_elems<BF16, TM>() + tile_elems<BF16, TN>()) * esz;
  static std::atomic<bool> done[kMaxDevices];
  const hipError_t e = once_per_device(done, [&] {
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&gemm_kernel<A_KC, B_KC, BF16, TM, TN, W32>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  });
  if (e != hipSuccess) return e;
  const int tiles = ((g.M + TM - 1) / TM) * ((g.N + TN - 1) / TN);
  hipLaunchKernelGGL((gemm_kernel<A_KC, B_KC, BF16, TM, TN, W32>), dim3(tiles, g.splits, g.batch > 1 ? g.batch : 1),
                     dim3(256), lds, s, g);
  return hipGetLastError();
}

template <bool A_KC, bool B_KC, bool BF16>
static hipError_t gemm_shape(GemmTile t, const GemmArgs& g, hipStream_t s) {
  switch (t) {
    case GEMM_TILE_32x128: return gemm_launch<A_KC, B_KC, BF16, 32, 128>(g, s);
    case GEMM_TILE_128x32: return gemm_launch<A_KC, B_KC, BF16, 128, 32>(g, s);
    case GEMM_TILE_128x64: return gemm_launch<A_KC, B_KC, BF16, 128, 64>(g, s);
    default:
      if (!BF16 && !g.mapped && g.splits == 1) return gemm_launch<A_KC, B_KC, BF16, 128, 128, true>(g, s);
      return gemm_launch<A_KC, B_KC, BF16, 128, 128>(g, s);
  }
}

int gemm_bk(bool bf16) { return bf16 ? GemmCfg<true>::BK : GemmCfg<false>::BK; }

GemmTile gemm_tile(int M, int N) {
  if (M <= 32 && N > 32) return GEMM_TILE_32x128;
  if (N <= 32) return GEMM_TILE_128x32;
  if (N <= 64) return GEMM_TILE_128x64;
  return GEMM_TILE_128x128;
}

void gemm_tile_dims(GemmTile t, int* tm, int* tn) {
  *tm = t == GEMM_TILE_32x128 ? 32 : 128;
  *tn = t == GEMM_TILE_128x32 ? 32 : (t == GEMM_TILE_128x64 ? 64 : 128);
}

hipError_t launch_gemm(bool a_kc, bool b_kc, bool bf16, const GemmArgs& g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  hipError_t e;
  const int idx = (a_kc ? 4 : 0) + (b_kc ? 2 : 0) + (bf16 ? 1 : 0);
  const GemmTile t = g.tile;
  switch (idx) {
    case 0: e = gemm_shape<false, false, false>(t, g, s); break;
    case 1: e = gemm_shape<false, false, true>(t, g, s); break;
    case 2: e = gemm_shape<false, true, false>(t, g, s); break;
    case 3: e = gemm_shape<false, true, true>(t, g, s); break;
    case 4: e = gemm_shape<true, false, false>(t, g, s); break;
    case 5: e = gemm_shape<true, false, true>(t, g, s); break;
    case 6: e = gemm_shape<true, true, false>(t, g, s); break;
    default: e = gemm_shape<true, true, true>(t, g, s); break;
  }
  if (e != hipSuccess || g.splits <= 1) return e;
  const long MN = (long)g.M * g.N;
  if (g.splits >= 256 && MN <= 65536)
    hipLaunchKernelGGL(splitk_reduce_kernel<64>, dim3((unsigned)((MN + 3) / 4)), dim3(256), 0, s, g.slab, g.splits,
                       g.M, g.N, g.alpha, g.C, g.ldc);
  else
    hipLaunchKernelGGL(splitk_reduce_kernel<8>, dim3((unsigned)((MN + 31) / 32)), dim3(256), 0, s, g.slab,
                       g.splits, g.M, g.N, g.alpha, g.C, g.ldc);
  return hipGetLastError();
}

hipError_t launch_gather(const GatherArgs& a, hipStream_t s) {
  if (a.M <= 0 || a.N <= 0) return hipSuccess;
  const IdxMap& mp = a.map;
  const bool vec = mp.ns0 == 1 && mp.nr0 % 4 == 0 && a.N % 4 == 0 && mp.ns1 % 4 == 0 && mp.ms0 % 4 == 0 &&
                   mp.ms1 % 4 == 0 && mp.ms2 % 4 == 0 && ((uintptr_t)a.src & 15) == 0 && ((uintptr_t)a.dst & 15) == 0;
  const long blocks = std::min<long>((a.M + 3) / 4, 16384);
  hipLaunchKernelGGL(gather_mapped_kernel, dim3((unsigned)blocks), dim3(256), 0, s, a, vec ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_core_perm(const float* src, float* dst, int R, int I, int J, int R1, int dir, hipStream_t s) {
  const long n = (long)R * I * J * R1;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(core_perm_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, dst, R, I, J, R1,
                     dir);
  return hipGetLastError();
}

hipError_t launch_tile_permute(const TilePermArgs& in, hipStream_t s) {
  if (in.tiles <= 0) return hipSuccess;
  TilePermArgs p = in;
  const int v = p.vec ? 4 : 1;
  p.fgp = make_fastdiv((uint32_t)(p.Bp / v));
  p.fgm = make_fastdiv((uint32_t)(p.Bm / v));
  p.fjl = make_fastdiv((uint32_t)p.Jl);
  const bool o16 = p.dir == 0 && p.dst16;
  const dim3 grid((unsigned)p.tiles);
  if (p.vec && o16)
    hipLaunchKernelGGL((tile_permute_kernel<4, true>), grid, dim3(256), 0, s, p);
  else if (p.vec)
    hipLaunchKernelGGL((tile_permute_kernel<4, false>), grid, dim3(256), 0, s, p);
  else if (o16)
    hipLaunchKernelGGL((tile_permute_kernel<1, true>), grid, dim3(256), 0, s, p);
  else
    hipLaunchKernelGGL((tile_permute_kernel<1, false>), grid, dim3(256), 0, s, p);
  return hipGetLastError();
}

hipError_t launch_permute(const PermArgs& p, hipStream_t s) {
  if (p.total <= 0) return hipSuccess;
  hipLaunchKernelGGL(permute_kernel, dim3((unsigned)((p.total + 255) / 256)), dim3(256), 0, s, p);
  return hipGetLastError();
}

int mse_blocks(long n) {
  long b = (n / 4 + 255) / 256;
  if (b < 1) b = 1;
  if (b > 2048) b = 2048;
  return (int)b;
}

hipError_t launch_mse(const float* y, const float* t, long n, float* dy, double* partials, double* out,
                      hipStream_t s) {
  const int nb = mse_blocks(n);
  hipLaunchKernelGGL(mse_partial_kernel, dim3(nb), dim3(256), 0, s, y, t, n, dy, 2.0 / (double)n, partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(mse_final_kernel, dim3(1), dim3(256), 0, s, partials, nb, 1.0 / (double)n, out);
  return hipGetLastError();
}

}  // namespace ttc
