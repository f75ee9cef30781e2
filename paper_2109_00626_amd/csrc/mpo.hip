// TT-matrix (MPO) x TT-vector on cores:
//   C^(k)[(a,r), i, (a',r')] = sum_j W^(k)[a, i, j, a'] V^(k)[r, j, r'].
// The output outnumbers the inputs by orders of magnitude (ranks multiply),
// so both kernels are streaming writers: each wave owns one (core, a, r) and
// writes the contiguous slab C[(a,r), i, :] of a1 x r1 values per mode index
// i, forming D_i[a', r'] = sum_j W[a, i, j, a'] V[r, j, r'] on 16x16 MFMA
// tiles (FP32 accumulation) and staging it through LDS so that every global
// store is 64 lanes x 16 contiguous bytes, non-temporal.
//
// mpo16_kernel (BF16 cores with J <= 64, r1 <= 128): a workgroup of waves
// with consecutive r shares one chunk of mode indices of W[a], staged once
// in LDS; each wave holds V[r] as MFMA operand fragments in registers, so
// its loop issues no global loads, only LDS reads, MFMAs and stores.
//
// mpo_stream_kernel (FP32 cores, and BF16 beyond those limits): one wave per
// (core, a, r), V staged in LDS as Vt[r'][j], and per mode index the slice
// W[a, i, :, :] as Wt[a'][j] (loaded four indices ahead into registers).
// Waves are independent (no barriers: LDS operations of one wave complete
// in order, and a compiler memory barrier keeps the staging writes and the
// differently typed operand reads in program order); LDS rows are padded
// with zeros to the MFMA's K step.
#include "ttc_device.hpp"
#include "ttc_internal.h"

#include <algorithm>

namespace ttc {

#define MPO_WAVES 4
#define MPO_PREF 8   // W elements per lane prefetched per index (the rest loads in place)
#define MPO_DEPTH 4  // indices of W prefetched ahead
#define MPO_COPY 8   // 16-byte output chunks per lane with precomputed LDS offsets

// Compiler-only memory barrier (no instruction): LDS written through one
// element type and read through another must not be reordered.
#define MPO_ORDER() asm volatile("" ::: "memory")

template <typename Tin>
struct MpoT;
template <>
struct MpoT<bf16_t> {
  typedef uint16_t E;
  static constexpr int KB = 32;  // K of one MFMA
  static constexpr int PAD = 8;  // LDS row padding (elements)
};
template <>
struct MpoT<float> {
  typedef float E;
  static constexpr int KB = 4;
  static constexpr int PAD = 4;
};

// Per-wave LDS layout of one core (elements of E, then floats).
struct MpoLds {
  int Jp, pitch, a1p, r1p, dp;
  long vt, wt, dl;  // byte offsets within the wave's region
  long bytes;
};
template <typename Tin>
__host__ __device__ inline MpoLds mpo_lds(int J, int a1, int r1) {
  typedef MpoT<Tin> T;
  MpoLds L;
  L.Jp = (J + T::KB - 1) / T::KB * T::KB;
  L.pitch = L.Jp + T::PAD;
  L.a1p = (a1 + 15) / 16 * 16;
  L.r1p = (r1 + 15) / 16 * 16;
  L.dp = L.r1p + 4;
  L.vt = 0;
  L.wt = L.vt + (long)L.r1p * L.pitch * (long)sizeof(typename T::E);
  L.wt = (L.wt + 15) & ~15L;
  L.dl = L.wt + (long)L.a1p * L.pitch * (long)sizeof(typename T::E);
  L.dl = (L.dl + 15) & ~15L;
  L.bytes = L.dl + (long)L.a1p * L.dp * 4 + 16;  // + a dummy slot for masked staging writes
  return L;
}

__device__ __forceinline__ const MpoCore& mpo_core_of(const MpoArgs& a, int item) {
  int c = 0;
  while (c + 1 < a.ncores && a.c[c + 1].blk_begin <= item) ++c;
  return a.c[c];
}

template <typename Tin>
__device__ __forceinline__ f32x4 mpo_tile(const typename MpoT<Tin>::E* Vt, const typename MpoT<Tin>::E* Wt, int pitch,
                                          int Jp, int rt, int at, int li, int g) {
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  if constexpr (sizeof(Tin) == 2) {
    for (int k0 = 0; k0 < Jp; k0 += 32) {
      const bf16x8 av = *reinterpret_cast<const bf16x8*>(Vt + (rt * 16 + li) * pitch + k0 + 8 * g);
      const bf16x8 bv = *reinterpret_cast<const bf16x8*>(Wt + (at * 16 + li) * pitch + k0 + 8 * g);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc, 0, 0, 0);
    }
  } else {
    for (int k0 = 0; k0 < Jp; k0 += 4) {
      const float av = Vt[(rt * 16 + li) * pitch + k0 + g];
      const float bv = Wt[(at * 16 + li) * pitch + k0 + g];
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc, 0, 0, 0);
    }
  }
  return acc;
}

// FIT: every core's W slice has at most 64 * MPO_PREF elements and every
// output row at most 256 * MPO_COPY, so the main loop has no loops of
// runtime length around memory operations (their unknown counts would force
// waits for every outstanding load and store).
template <typename Tin, bool FIT>
__global__ __launch_bounds__(64 * MPO_WAVES) void mpo_stream_kernel(MpoArgs a, int wave_bytes) {
  typedef typename MpoT<Tin>::E E;
  extern __shared__ __align__(16) unsigned char smem[];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform per wave
  const int li = lane & 15, g = lane >> 4;
  const int item = blockIdx.x * MPO_WAVES + wave;
  if (item >= a.nblk) return;  // whole waves only: no barriers follow
  const MpoCore& c = mpo_core_of(a, item);
  const int local = item - c.blk_begin;
  const int aa = local / c.r0, r = local - aa * c.r0;
  const int I = c.I, J = c.J, a1 = c.a1, r1 = c.r1;
  const MpoLds L = mpo_lds<Tin>(J, a1, r1);
  unsigned char* base = smem + (long)wave * wave_bytes;
  E* Vt = reinterpret_cast<E*>(base + L.vt);
  E* Wt = reinterpret_cast<E*>(base + L.wt);
  float* Dl = reinterpret_cast<float*>(base + L.dl);
  const E* Vg = reinterpret_cast<const E*>(c.v) + (long)r * J * r1;
  const E* Wg = reinterpret_cast<const E*>(c.w) + (long)aa * I * J * a1;
  float* out = reinterpret_cast<float*>(c.out) + (long)(aa * c.r0 + r) * I * a1 * r1;
  // zero both staging tiles (padding stays zero), then V[r] as Vt[r'][j]
  for (int e = lane; e < L.r1p * L.pitch; e += 64) Vt[e] = (E)0;
  for (int e = lane; e < L.a1p * L.pitch; e += 64) Wt[e] = (E)0;
  for (int e = lane; e < J * r1; e += 64) {
    const int j = e / r1, rp = e - j * r1;
    Vt[rp * L.pitch + j] = Vg[e];
  }
  MPO_ORDER();
  const int JA = J * a1;
  // W slices run MPO_DEPTH indices ahead in a register ring (the loop below
  // is unrolled by MPO_DEPTH so every slot index is static); the LDS offsets
  // of the prefetched elements are the same for every index
  E pf[MPO_DEPTH][MPO_PREF];
  int woff[MPO_PREF];
  // (elements past the slice load a valid address and land in a dummy LDS
  // slot, so staging has no branches and no early waits)
  const int dummy = (int)((L.dl + (long)L.a1p * L.dp * 4 - L.wt) / (long)sizeof(E));
  int eoff[MPO_PREF];
#pragma unroll
  for (int t = 0; t < MPO_PREF; ++t) {
    const int e = lane + 64 * t;
    const int j = e / a1, ap = e - j * a1;
    woff[t] = (e < JA) ? ap * L.pitch + j : dummy;
    eoff[t] = min(e, JA - 1);
  }
#pragma unroll
  for (int d = 0; d < MPO_DEPTH; ++d)
#pragma unroll
    for (int t = 0; t < MPO_PREF; ++t) pf[d][t] = Wg[(long)min(d, I - 1) * JA + eoff[t]];
  const int RT = L.r1p / 16, AT = L.a1p / 16;
  const int n = a1 * r1;
  const bool vec = (r1 % 4 == 0) && ((reinterpret_cast<uintptr_t>(out) & 15) == 0);
  // LDS offsets of the lane's copy-out chunks (vector path, first MPO_COPY)
  int doff[MPO_COPY];
#pragma unroll
  for (int q = 0; q < MPO_COPY; ++q) {
    const int e = 4 * lane + 256 * q;
    const int ap = e / r1, rp = e - ap * r1;
    doff[q] = ap * L.dp + rp;
  }
  for (int i0 = 0; i0 < I; i0 += MPO_DEPTH) {
#pragma unroll
    for (int d = 0; d < MPO_DEPTH; ++d) {
      const int i = i0 + d;
      if (i >= I) break;
      // W[a, i] into Wt[a'][j]: the prefetched part, then any remainder
#pragma unroll
      for (int t = 0; t < MPO_PREF; ++t) Wt[woff[t]] = pf[d][t];
      if constexpr (!FIT)
        for (int e = lane + 64 * MPO_PREF; e < JA; e += 64) {
          const int j = e / a1, ap = e - j * a1;
          Wt[ap * L.pitch + j] = Wg[(long)i * JA + e];
        }
      MPO_ORDER();
      if (i + MPO_DEPTH < I) {
        const E* src = Wg + (long)(i + MPO_DEPTH) * JA;
#pragma unroll
        for (int t = 0; t < MPO_PREF; ++t) pf[d][t] = src[eoff[t]];
      }
      // D_i tiles -> Dl[a'][r']
      for (int at = 0; at < AT; ++at)
        for (int rt = 0; rt < RT; ++rt) {
          const f32x4 acc = mpo_tile<Tin>(Vt, Wt, L.pitch, L.Jp, rt, at, li, g);
          *reinterpret_cast<f32x4*>(Dl + (at * 16 + li) * L.dp + rt * 16 + 4 * g) = acc;
        }
      MPO_ORDER();
      // contiguous copy-out of the a1 x r1 block of index i
      float* orow = out + (long)i * n;
      if (vec) {
#pragma unroll
        for (int q = 0; q < MPO_COPY; ++q) {
          const int e = 4 * lane + 256 * q;
          if (e < n)
            __builtin_nontemporal_store(*reinterpret_cast<const f32x4*>(Dl + doff[q]),
                                        reinterpret_cast<f32x4*>(orow + e));
        }
        if constexpr (!FIT)
          for (int e = 4 * lane + 256 * MPO_COPY; e < n; e += 256) {
            const int ap = e / r1, rp = e - ap * r1;
            const f32x4 v = *reinterpret_cast<const f32x4*>(Dl + ap * L.dp + rp);
            __builtin_nontemporal_store(v, reinterpret_cast<f32x4*>(orow + e));
          }
      } else if constexpr (FIT) {
#pragma unroll
        for (int q = 0; q < 4 * MPO_COPY; ++q) {
          const int e = lane + 64 * q;
          if (e < n) {
            const int ap = e / r1, rp = e - ap * r1;
            __builtin_nontemporal_store(Dl[ap * L.dp + rp], orow + e);
          }
        }
      } else {
        for (int e = lane; e < n; e += 64) {
          const int ap = e / r1, rp = e - ap * r1;
          __builtin_nontemporal_store(Dl[ap * L.dp + rp], orow + e);
        }
      }
      MPO_ORDER();
    }
  }
}

// BF16 inputs, a workgroup per (core, a, group of MPO16_WAVES consecutive
// r, chunk of MPO16_CHUNK mode indices i).  The workgroup stages its chunk
// of W[a] in LDS as Ws[i][a'][j] (zero-padded), shared by its waves; each
// wave keeps V[r] as MFMA operand fragments (r' on the operand's rows, j on
// its K), so the loop reads one LDS fragment per 16 values of a' and issues
// no global loads, hence no waits on the stores in flight.  A lane's
// accumulator holds four consecutive r' of one a'; a wave's 16 rows a' of
// one index are one contiguous run of the output, written through a
// wave-private staging tile.  Chunks of 4 indices and 8 waves: 0.161 ms on
// the order-8 rank-16 x rank-64 product (0.174 ms with chunks of 8, 0.237
// ms with 1; the register-prefetching kernel above, 0.180 ms).
#ifndef MPO16_WAVES
#define MPO16_WAVES 8
#endif
#ifndef MPO16_CHUNK
#define MPO16_CHUNK 4
#endif

// LDS row pitch of Ws (BF16 elements) for KT 32-wide K steps
__host__ __device__ inline int mpo16_pitch(int kt) { return kt * 32 + 8; }

// Groups of MPO16_WAVES consecutive vector bonds r of one core.
__host__ __device__ inline int mpo16_groups(const MpoCore& c) { return (c.r0 + MPO16_WAVES - 1) / MPO16_WAVES; }

// KT: 32-wide K steps (J <= 32 KT); RTM: r' tiles held in registers
// (r1 <= 16 RTM), all computed (zero fragments past r1), stored where valid.
template <int KT, int RTM>
__global__ __launch_bounds__(64 * MPO16_WAVES) void mpo16_kernel(MpoArgs a, int ic, int ws_bytes) {
  extern __shared__ __align__(16) unsigned char smem[];
  uint16_t* Ws = reinterpret_cast<uint16_t*>(smem);
  const MpoCore& c = mpo_core_of(a, blockIdx.x);
  const int I = c.I, J = c.J, a1 = c.a1, r1 = c.r1, r0 = c.r0;
  const int nh = (I + ic - 1) / ic, ng = mpo16_groups(c);
  const int local = blockIdx.x - c.blk_begin;
  const int aa = local / (ng * nh), rem = local - aa * (ng * nh);
  const int grp = rem / nh, h = rem - grp * nh;
  const int i0 = h * ic, icn = min(ic, I - i0);
  const int a1p = (a1 + 15) / 16 * 16, pitch = mpo16_pitch(KT);
  const int lane = threadIdx.x & 63, li = lane & 15, g = lane >> 4;
  const int wave = threadIdx.x >> 6;
  // W[a, i0 .. i0+icn) -> Ws[ii][a'][j]: the data (contiguous in W), then
  // the padding (a' >= a1 or j >= J), disjoint LDS locations
  const uint16_t* Wg = reinterpret_cast<const uint16_t*>(c.w) + ((long)aa * I + i0) * J * a1;
  const int JA = J * a1, tot = icn * JA;
  for (int e = threadIdx.x; e < tot; e += 64 * MPO16_WAVES) {
    const int ii = e / JA, q = e - ii * JA;
    const int j = q / a1, ap = q - j * a1;
    Ws[(ii * a1p + ap) * pitch + j] = Wg[e];
  }
  const int lds_e = icn * a1p * pitch;
  for (int e = threadIdx.x; e < lds_e; e += 64 * MPO16_WAVES) {
    const int row = e / pitch, j = e - row * pitch;
    const int ap = row % a1p;
    if (ap >= a1 || j >= J) Ws[e] = 0;
  }
  // the wave's V[r] as operand fragments: lane (li, g) of fragment (rt, kt)
  // holds V[r, kt*32 + 8g + t, rt*16 + li], t = 0..7
  const int r = grp * MPO16_WAVES + wave;
  const int AT = a1p / 16;
  uint4 Af[RTM][KT];
  if (r < r0) {
    // every load is issued (clamped into the core), then the out-of-range
    // elements are zeroed, so the loads overlap
    const uint16_t* Vg = reinterpret_cast<const uint16_t*>(c.v) + (long)r * J * r1;
    uint16_t x[RTM][KT][8];
#pragma unroll
    for (int rt = 0; rt < RTM; ++rt)
#pragma unroll
      for (int kt = 0; kt < KT; ++kt)
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          const int rp = min(rt * 16 + li, r1 - 1), j = min(kt * 32 + 8 * g + t, J - 1);
          x[rt][kt][t] = Vg[(long)j * r1 + rp];
        }
#pragma unroll
    for (int rt = 0; rt < RTM; ++rt)
#pragma unroll
      for (int kt = 0; kt < KT; ++kt) {
        uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          const bool ok = rt * 16 + li < r1 && kt * 32 + 8 * g + t < J;
          w[t >> 1] |= (ok ? (uint32_t)x[rt][kt][t] : 0u) << (16 * (t & 1));
        }
        Af[rt][kt] = make_uint4(w[0], w[1], w[2], w[3]);
      }
  }
  __syncthreads();
  if (r >= r0) return;  // no barriers follow
  const int n = a1 * r1;
  const bool vec = (r1 % 4 == 0) && ((reinterpret_cast<uintptr_t>(c.out) & 15) == 0);
  float* out = reinterpret_cast<float*>(c.out) + ((long)(aa * r0 + r) * I + i0) * n;
  // the wave's staging tile: 16 rows a' of up to 16 RTM values r'
  constexpr int DP = 16 * RTM + 4;
  float* Dl = reinterpret_cast<float*>(smem + ws_bytes) + wave * 16 * DP;
  // staging offsets of the lane's 16-byte chunks of a 16 x r1 run (at most
  // 256 RTM values: RTM chunks per lane)
  int doff[RTM];
#pragma unroll
  for (int q = 0; q < RTM; ++q) {
    const int e = 4 * lane + 256 * q;
    doff[q] = (e / r1) * DP + e % r1;
  }
  for (int ii = 0; ii < icn; ++ii) {
    float* orow = out + (long)ii * n;
    for (int at = 0; at < AT; ++at) {
      uint4 B[KT];
#pragma unroll
      for (int kt = 0; kt < KT; ++kt)
        B[kt] = *reinterpret_cast<const uint4*>(Ws + (ii * a1p + at * 16 + li) * pitch + kt * 32 + 8 * g);
      f32x4 acc[RTM];
#pragma unroll
      for (int rt = 0; rt < RTM; ++rt) {
        acc[rt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kt = 0; kt < KT; ++kt)
          acc[rt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, Af[rt][kt]),
                                                            __builtin_bit_cast(bf16x8, B[kt]), acc[rt], 0, 0, 0);
      }
      if (vec) {
        // rows a' = at*16 .. are one contiguous run of the output: through
        // the staging tile, 64 lanes x 16 consecutive bytes per store (the
        // accumulators stored directly write 64-byte runs of four lanes:
        // half of each 128-byte line per instruction, measured at half the
        // rate)
#pragma unroll
        for (int rt = 0; rt < RTM; ++rt) *reinterpret_cast<f32x4*>(Dl + li * DP + rt * 16 + 4 * g) = acc[rt];
        MPO_ORDER();
        const int m = min(16, a1 - at * 16) * r1;
        float* o = orow + (long)at * 16 * r1;
#pragma unroll
        for (int q = 0; q < RTM; ++q) {
          const int e = 4 * lane + 256 * q;
          if (e < m)
            __builtin_nontemporal_store(*reinterpret_cast<const f32x4*>(Dl + doff[q]),
                                        reinterpret_cast<f32x4*>(o + e));
        }
        MPO_ORDER();
        continue;
      }
      const int ap = at * 16 + li;
#pragma unroll
      for (int rt = 0; rt < RTM; ++rt) {
        const int rp = rt * 16 + 4 * g;
        float* p = orow + ap * r1 + rp;
        if (vec) {
          if (ap < a1 && rp < r1) __builtin_nontemporal_store(acc[rt], reinterpret_cast<f32x4*>(p));
        } else {
#pragma unroll
          for (int v = 0; v < 4; ++v)
            if (ap < a1 && rp + v < r1) __builtin_nontemporal_store(acc[rt][v], p + v);
        }
      }
    }
  }
}

// The register-fragment kernel takes BF16 cores with J <= 64 and r1 <= 128;
// the mode-index chunk shrinks until its LDS fits.  Returns false when the
// shapes are beyond it.
static bool launch_mpo16(MpoArgs a, hipStream_t s, hipError_t* err) {
  int kt = 1, rtm = 4;
  for (int k = 0; k < a.ncores; ++k) {
    const MpoCore& c = a.c[k];
    if (c.J > 64 || c.r1 > 128) return false;
    if (c.J > 32) kt = 2;
    if (c.r1 > 64) rtm = 8;
  }
  const long cap = 80 * 1024;
  const long dl = (long)MPO16_WAVES * 16 * (16 * rtm + 4) * 4;
  int ic = MPO16_CHUNK;
  long ws = 0;
  for (;;) {
    ws = 0;
    for (int k = 0; k < a.ncores; ++k) {
      const MpoCore& c = a.c[k];
      ws = std::max(ws, (long)std::min(ic, c.I) * ((c.a1 + 15) / 16 * 16) * mpo16_pitch(kt) * 2);
    }
    ws = (ws + 15) & ~15L;
    if (ws + dl <= cap || ic == 1) break;
    ic /= 2;
  }
  const long lds = ws + dl;
  if (lds > cap) return false;
  long blocks = 0;
  for (int k = 0; k < a.ncores; ++k) {
    MpoCore& c = a.c[k];
    c.blk_begin = (int)blocks;
    blocks += (long)c.a0 * mpo16_groups(c) * ((c.I + ic - 1) / ic);
  }
  if (blocks > 0x7fffffffL) return false;
  a.nblk = (int)blocks;
  if (blocks == 0) {
    *err = hipSuccess;
    return true;
  }
  const void* fn = kt == 1 ? (rtm == 4 ? reinterpret_cast<const void*>(&mpo16_kernel<1, 4>)
                                       : reinterpret_cast<const void*>(&mpo16_kernel<1, 8>))
                           : (rtm == 4 ? reinterpret_cast<const void*>(&mpo16_kernel<2, 4>)
                                       : reinterpret_cast<const void*>(&mpo16_kernel<2, 8>));
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e == hipSuccess) {
    const dim3 grid((unsigned)blocks), block(64 * MPO16_WAVES);
    if (kt == 1 && rtm == 4)
      hipLaunchKernelGGL((mpo16_kernel<1, 4>), grid, block, (size_t)lds, s, a, ic, (int)ws);
    else if (kt == 1)
      hipLaunchKernelGGL((mpo16_kernel<1, 8>), grid, block, (size_t)lds, s, a, ic, (int)ws);
    else if (rtm == 4)
      hipLaunchKernelGGL((mpo16_kernel<2, 4>), grid, block, (size_t)lds, s, a, ic, (int)ws);
    else
      hipLaunchKernelGGL((mpo16_kernel<2, 8>), grid, block, (size_t)lds, s, a, ic, (int)ws);
    e = hipGetLastError();
  }
  *err = e;
  return true;
}

// Any dtype, plain FMA: one thread per output entry.
template <typename Tin, typename Tc>
__global__ __launch_bounds__(256) void mpo_generic_kernel(MpoArgs a) {
  const MpoCore& c = mpo_core_of(a, blockIdx.x);
  const long per = (long)c.a0 * c.r0 * c.I * c.a1 * c.r1;
  const long e = (long)(blockIdx.x - c.blk_begin) * blockDim.x + threadIdx.x;
  if (e >= per) return;
  const int d1 = c.a1 * c.r1;
  const int col = (int)(e % d1);
  const long ri = e / d1;
  const int i = (int)(ri % c.I);
  const int row = (int)(ri / c.I);
  const int aa = row / c.r0, r = row - aa * c.r0;
  const int ap = col / c.r1, rp = col - ap * c.r1;
  const Tin* W = reinterpret_cast<const Tin*>(c.w) + (((long)aa * c.I + i) * c.J) * c.a1 + ap;
  const Tin* V = reinterpret_cast<const Tin*>(c.v) + (long)r * c.J * c.r1 + rp;
  Tc acc = 0;
  for (int j = 0; j < c.J; ++j) acc += cvt<Tc>(W[(long)j * c.a1]) * cvt<Tc>(V[(long)j * c.r1]);
  reinterpret_cast<Tc*>(c.out)[e] = acc;
}

// Per-wave LDS bytes of the streaming kernel for the largest core.
template <typename Tin>
long mpo_wave_bytes(const MpoArgs& a) {
  long mx = 0;
  for (int k = 0; k < a.ncores; ++k) mx = std::max(mx, mpo_lds<Tin>(a.c[k].J, a.c[k].a1, a.c[k].r1).bytes);
  return (mx + 15) & ~15L;
}

template <typename Tin, bool FIT>
hipError_t launch_mpo_stream_as(const MpoArgs& a, int items, long wb, hipStream_t s) {
  const int lds = (int)(wb * MPO_WAVES);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&mpo_stream_kernel<Tin, FIT>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((mpo_stream_kernel<Tin, FIT>), dim3((items + MPO_WAVES - 1) / MPO_WAVES), dim3(64 * MPO_WAVES),
                     (size_t)lds, s, a, (int)wb);
  return hipGetLastError();
}

template <typename Tin>
hipError_t launch_mpo_stream(MpoArgs a, hipStream_t s) {
  const long wb = mpo_wave_bytes<Tin>(a);
  int items = 0;
  bool fit = true;
  for (int k = 0; k < a.ncores; ++k) {
    a.c[k].blk_begin = items;
    items += a.c[k].a0 * a.c[k].r0;
    fit = fit && a.c[k].J * a.c[k].a1 <= 64 * MPO_PREF && a.c[k].a1 * a.c[k].r1 <= 256 * MPO_COPY;
  }
  a.nblk = items;
  if (items <= 0) return hipSuccess;
  return fit ? launch_mpo_stream_as<Tin, true>(a, items, wb, s) : launch_mpo_stream_as<Tin, false>(a, items, wb, s);
}

hipError_t launch_mpo(ttc_dtype dt, bool bf16_mfma, const MpoArgs& in, hipStream_t s) {
  (void)bf16_mfma;  // BF16 inputs always use BF16 MFMA with FP32 accumulation
  hipError_t err16;
  if (dt == TTC_BF16 && launch_mpo16(in, s, &err16)) return err16;
  if (dt == TTC_BF16 && mpo_wave_bytes<bf16_t>(in) * MPO_WAVES <= lds_limit_bytes())
    return launch_mpo_stream<bf16_t>(in, s);
  if (dt == TTC_F32 && mpo_wave_bytes<float>(in) * MPO_WAVES <= lds_limit_bytes())
    return launch_mpo_stream<float>(in, s);
  MpoArgs a = in;
  int nblk = 0;
  for (int k = 0; k < a.ncores; ++k) {
    MpoCore& c = a.c[k];
    c.blk_begin = nblk;
    const long per = (long)c.a0 * c.r0 * c.I * c.a1 * c.r1;
    nblk += (int)((per + 255) / 256);
  }
  a.nblk = nblk;
  if (nblk <= 0) return hipSuccess;
  switch (dt) {
    case TTC_F64: hipLaunchKernelGGL((mpo_generic_kernel<double, double>), dim3(nblk), dim3(256), 0, s, a); break;
    case TTC_F32: hipLaunchKernelGGL((mpo_generic_kernel<float, float>), dim3(nblk), dim3(256), 0, s, a); break;
    default: hipLaunchKernelGGL((mpo_generic_kernel<bf16_t, float>), dim3(nblk), dim3(256), 0, s, a); break;
  }
  return hipGetLastError();
}

}  // namespace ttc
