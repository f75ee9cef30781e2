// Interface sweep step for BF16 cores on BF16 MFMA, FP32 accumulation.
//
// The step is that of sweep_lds.hpp,
//   Out[a, b] = sum_i sum_{a', b'} G_A[a, i, a'] In[a', b'] G_B[b, i, b'],
// as two chained products per mode index (S_i^T = In^T G_A[:, i, :]^T, then
// Out += S_i G_B[:, i, :]^T), but on the 16x16x32 BF16 MFMA, which needs
// BF16 operands on both sides.  The
// cores are BF16 already.  The interface In and the per-index product S_i
// are FP32 sums; each is carried as a pair of BF16 values, hi = bf16(v) and
// lo = bf16(v - hi) (16 significant bits; integers below 2^16 stay exact),
// and each product with a core is two MFMAs, hi and lo, into one FP32
// accumulator.  Against FP32 operands this is 2 x 16 cycles of matrix core
// per 16 x 16 x 32 block instead of 8 x 32.
//
// The interface lives in LDS as two planes of BF16, hi at `In` and lo at
// `In + lo`, zero-padded to multiples of 16 like the FP32 layout, with rows
// of lds16_pitch(n) = pad16(n) + 8 elements (a byte stride of 16 x odd, so 16
// lanes reading 16 bytes from 16 consecutive rows touch disjoint banks).
// A step splits its FP32 output tiles into the two planes once, in the
// orientation the next step reads.
//
// K index order inside an MFMA operand (any order works as long as both
// operands use it): along a' a 32-wide chunk c gives lane group g the eight
// consecutive a' = 32c + 8g + j; along b' a 32-wide block q gives it
// b' = 32q + 4g + j (j < 4) and 32q + 16 + 4g + (j - 4), the rows the two
// stage-1 tiles of the block leave in that lane's accumulators.  A trailing
// 16-wide chunk of a' (or block of b') runs as a 32-wide product whose slots
// j >= 4 are zero in both operands, lane group g holding a' = 32c + 4g + j
// (b' = 32q + 4g + j) in slots j < 4.  Every accumulator chain thus uses one
// MFMA kind only: a 16x16x16 product reading a 16x16x32 product's result as
// its accumulator gave wrong sums on gfx950 without added wait states.
#pragma once
#include "sweep_lds.hpp"


namespace ttc {

__host__ __device__ __forceinline__ int lds16_pitch(int n) { return pad16(n) + 8; }

// BF16 elements of one plane able to hold R x P in either layout (the two
// planes together take as many bytes as that many floats).
__host__ __device__ __forceinline__ int lds16_iface_elems(int R, int P) {
  const int t = pad16(P) * lds16_pitch(R), n = pad16(R) * lds16_pitch(P);
  return t > n ? t : n;
}

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ f32x4 mfma_b32(const uint4& a, const uint4& b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0,
                                                 0, 0);
}
// 32-wide product of four BF16 values per lane (slots 4..7 zero)
__device__ __forceinline__ f32x4 mfma_b32h(const uint2& a, const uint2& b, f32x4 c) {
  return mfma_b32(make_uint4(a.x, a.y, 0u, 0u), make_uint4(b.x, b.y, 0u, 0u), c);
}

// Two FP32 values to packed BF16 (element 0 in the low half), round to
// nearest even.
__device__ __forceinline__ unsigned pk_bf16(float a, float b) {
  const f32x2 v = {a, b};
  return __builtin_bit_cast(unsigned, __builtin_convertvector(v, bf16x2));
}
__device__ __forceinline__ float bf16_lo(unsigned w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16_hi(unsigned w) { return __uint_as_float(w & 0xFFFF0000u); }

// hi / lo split of two FP32 values: packed hi = bf16(v), lo = bf16(v - hi).
__device__ __forceinline__ void split2(float a, float b, unsigned& h, unsigned& l) {
  h = pk_bf16(a, b);
  l = pk_bf16(a - bf16_lo(h), b - bf16_hi(h));
}

// Mask keeping element j of four consecutive BF16 elements e0 + j when e0 + j < K.
__device__ __forceinline__ uint2 keep4(int e0, int K) {
  return make_uint2((e0 < K ? 0xFFFFu : 0u) | (e0 + 1 < K ? 0xFFFF0000u : 0u),
                    (e0 + 2 < K ? 0xFFFFu : 0u) | (e0 + 3 < K ? 0xFFFF0000u : 0u));
}
__device__ __forceinline__ uint2 and2(const uint2& v, const uint2& m) { return make_uint2(v.x & m.x, v.y & m.y); }
__device__ __forceinline__ uint4 cat2(const uint2& a, const uint2& b) { return make_uint4(a.x, a.y, b.x, b.y); }

typedef unsigned u32x3 __attribute__((ext_vector_type(3)));
typedef unsigned u32x4_t __attribute__((ext_vector_type(4)));

// Three dwords of a core at a dword-aligned byte offset (zeros past the
// resource's end).
__device__ __forceinline__ u32x3 raw_at(const CoreRes& c, int off) {
  return __builtin_amdgcn_raw_buffer_load_b96(c.r, off, 0, 0);
}
// Four BF16 elements starting `sh` bits into the three dwords.
__device__ __forceinline__ uint2 take_raw(const u32x3& v, int sh) {
  return make_uint2(__builtin_amdgcn_alignbit(v[1], v[0], sh), __builtin_amdgcn_alignbit(v[2], v[1], sh));
}

// Mode indices per loop trip: the BF16 products are cheap, so every shape
// with room in the register file takes several.
template <int KC, int PT>
struct TripWidth16 {
  static constexpr int U = (KC + PT <= 4) ? 4 : (KC + PT <= 6) ? 2 : 1;
};

// A rough count of the VGPRs a trip holds for NA a-tiles and U mode
// indices: accumulators, the larger of the G_A operands and their raw
// reload, the raw G_B loads with the operands shifted out of them, the
// stage-1 tiles.  The bound it is compared with was chosen by timing.
template <int KC, int PT, int NA, int U>
struct TripRegs {
  static constexpr int KP = KC / 2, KT = KC & 1;
  static constexpr int ga = NA * U * (KP * 4 + KT * 2), gar = NA * U * (KP * 6 + KT * 3);
  static constexpr int n = NA * PT * 4 + (ga > gar ? ga : gar) + U * PT * (8 + 6 * 2) / 2 + NA * U * 8;
};

// Accumulate mode indices i = s0, s0 + S, ... into NA a-tiles (at[0], and
// at[1] when NA == 2) of Out.  KC = pad16(Ka) / 16, PT = pad16(Nb) / 16.  A
// loop trip covers U mode indices (those past I read zeros through empty
// resources) and one 32-wide block q of b' (the last block is 16 wide when
// pad16(Kb) is an odd multiple of 16).  The G_A rows of the next mode
// indices are loaded right after this trip's stage-1 products (their last
// use) and shifted into operands at the end of the trip; the G_B rows of the
// next block after this trip's stage-2 products, shifted into operands as
// that block's stage 2 uses them.  Core entries past a row's end (the next
// entries of the core) are masked to zero.
template <int KC, int PT, int NA, int U>
__device__ __forceinline__ void lds16_tiles(const StepOp& op, const TTC_LDS uint16_t* __restrict__ In, int lo,
                                            const int (&at)[2], int s0, int S, f32x4 (&acc0)[SW_MAXT],
                                            f32x4 (&acc1)[SW_MAXT]) {
  constexpr int KP = KC / 2, KT = KC & 1, KPA = KP > 0 ? KP : 1;
  const int lane = threadIdx.x & 63, li = lane & 15, g = lane >> 4;
  const int I = __builtin_amdgcn_readfirstlane(op.I), Ka = __builtin_amdgcn_readfirstlane(op.Ka),
            Kb = __builtin_amdgcn_readfirstlane(op.Kb);
  const int QT = (Kb + 15) >> 4, QB = (QT + 1) >> 1;
  const int ip = lds16_pitch(Ka);
  const long ta = (long)op.Ma * I * Ka, tb = (long)op.Nb * I * Kb;
  // Per-lane byte offsets of the core rows, split into a dword-aligned part
  // and the row's 2-byte parity (the same for every chunk and tile of the
  // lane); a resource adds its own parity `adj`, and the sum picks the dword
  // to load and the funnel shift (see raw_at / take_raw).
  int aal[NA];
#pragma unroll
  for (int t = 0; t < NA; ++t) aal[t] = ((at[t] * 16 + li) * I * Ka * 2) & ~3;
  const int apar = ((li * I * Ka) & 1) << 1;
  int bal[PT];
#pragma unroll
  for (int pt = 0; pt < PT; ++pt) bal[pt] = (((pt * 16 + li) * I * Kb + 4 * g) * 2) & ~3;
  const int bpar = ((li * I * Kb) & 1) << 1;
  // masks of the last chunk along a' when it is partial
  const bool apart = (Ka & 15) != 0;
  const uint2 ma0 = KT ? keep4(32 * KP + 4 * g, Ka) : keep4(32 * (KP - 1) + 8 * g, Ka);
  const uint2 ma1 = keep4(32 * (KP - 1) + 8 * g + 4, Ka);
  if (s0 >= I) return;
  const int step = U * S;

  // Loads keep the raw dwords; the funnel shift happens when the operands
  // are taken, so no load is waited for inside the (conditional) code that
  // issues it.
  uint4 ga[NA][U][KPA];
  uint2 gat[NA][U];
  u32x3 gar[NA][U][KPA][2], gatr[NA][U];
  int sha[U];
  // G_B rows of the current block, raw: b' = 32q + 4g + j and 32q + 16 + 4g + j
  u32x3 gr0[U][PT], gr1[U][PT];
  int shb[U];

  auto load_a = [&](int i0) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const CoreRes ra = core_rsrc_if(i0 + u * S < I, op.ga, (long)(i0 + u * S) * Ka, ta, 2);
      const int corr = (apar & ra.adj) << 1;
      sha[u] = (apar ^ ra.adj) << 3;
#pragma unroll
      for (int t = 0; t < NA; ++t) {
        const int o = aal[t] + corr;
#pragma unroll
        for (int c = 0; c < KP; ++c) {
          gar[t][u][c][0] = raw_at(ra, o + (32 * c + 8 * g) * 2);
          gar[t][u][c][1] = raw_at(ra, o + (32 * c + 8 * g + 4) * 2);
        }
        if constexpr (KT) gatr[t][u] = raw_at(ra, o + (32 * KP + 4 * g) * 2);
      }
    }
  };
  // the loaded G_A rows as operands, masked past the row ends
  auto take_a = [&]() {
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int t = 0; t < NA; ++t) {
#pragma unroll
        for (int c = 0; c < KP; ++c)
          ga[t][u][c] = cat2(take_raw(gar[t][u][c][0], sha[u]), take_raw(gar[t][u][c][1], sha[u]));
        if constexpr (KT) gat[t][u] = take_raw(gatr[t][u], sha[u]);
      }
    if (!apart) return;
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int t = 0; t < NA; ++t) {
        if constexpr (KT) {
          gat[t][u] = and2(gat[t][u], ma0);
        } else {
          uint4& v = ga[t][u][KP - 1];
          v = make_uint4(v.x & ma0.x, v.y & ma0.y, v.z & ma1.x, v.w & ma1.y);
        }
      }
  };
  // G_B rows of block q for mode indices i0 + u S (both halves; those past
  // the core read zeros, the rest of a half block is never used)
  auto load_b = [&](int i0, int q) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const CoreRes rb = core_rsrc_if(i0 + u * S < I, op.gb, (long)(i0 + u * S) * Kb + 32 * q, tb, 2);
      const int corr = (bpar & rb.adj) << 1;
      shb[u] = (bpar ^ rb.adj) << 3;
#pragma unroll
      for (int pt = 0; pt < PT; ++pt) {
        gr0[u][pt] = raw_at(rb, bal[pt] + corr);
        gr1[u][pt] = raw_at(rb, bal[pt] + corr + 32);
      }
    }
  };

  load_a(s0);
  load_b(s0, 0);
  take_a();
  __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
  int i = s0, q = 0;
  for (;;) {
    int ni = i, nq = q + 1;
    if (nq == QB) {
      nq = 0;
      ni = i + step;
    }
    const bool more = ni < I;
    const bool full = 2 * q + 1 < QT;
    // stage 1: S^T rows b' = 32q + 16h + (0..15) of each tile and mode index
    f32x4 st[NA][U][2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (h == 1 && !full) break;
      const TTC_LDS uint16_t* row = In + (32 * q + 16 * h + li) * ip;
#pragma unroll
      for (int t = 0; t < NA; ++t)
#pragma unroll
        for (int u = 0; u < U; ++u) st[t][u][h] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int c = 0; c < KP; ++c) {
        const uint4 vh = *reinterpret_cast<const TTC_LDS uint4*>(row + 32 * c + 8 * g);
        const uint4 vl = *reinterpret_cast<const TTC_LDS uint4*>(row + lo + 32 * c + 8 * g);
#pragma unroll
        for (int t = 0; t < NA; ++t)
#pragma unroll
          for (int u = 0; u < U; ++u) {
            st[t][u][h] = mfma_b32(vh, ga[t][u][c], st[t][u][h]);
            st[t][u][h] = mfma_b32(vl, ga[t][u][c], st[t][u][h]);
          }
      }
      if constexpr (KT) {
        const uint2 vh = *reinterpret_cast<const TTC_LDS uint2*>(row + 32 * KP + 4 * g);
        const uint2 vl = *reinterpret_cast<const TTC_LDS uint2*>(row + lo + 32 * KP + 4 * g);
#pragma unroll
        for (int t = 0; t < NA; ++t)
#pragma unroll
          for (int u = 0; u < U; ++u) {
            st[t][u][h] = mfma_b32h(vh, gat[t][u], st[t][u][h]);
            st[t][u][h] = mfma_b32h(vl, gat[t][u], st[t][u][h]);
          }
      }
    }
    // the next mode indices' G_A rows (this trip's stage 1 was their last use)
    const bool reload = more && nq == 0;
    if (reload) load_a(ni);
    // stage 2: Out[a-tile, b-tile pt] += S_i[:, block q] . G_B[b-tile, i, block q]^T,
    // the G_B operands shifted out of the raw loads (masked past Kb in a last
    // partial block)
    const bool bpart = 32 * q + 32 > Kb;
    const uint2 m0 = keep4(32 * q + 4 * g, Kb), m1 = keep4(32 * q + 16 + 4 * g, Kb);
    auto gbop = [&](int u, int pt, bool second) -> uint2 {
      uint2 v = take_raw(second ? gr1[u][pt] : gr0[u][pt], shb[u]);
      if (bpart) v = and2(v, second ? m1 : m0);
      return v;
    };
#pragma unroll
    for (int t = 0; t < NA; ++t)
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (full) {
          unsigned h0, l0, h1, l1, h2, l2, h3, l3;
          split2(st[t][u][0][0], st[t][u][0][1], h0, l0);
          split2(st[t][u][0][2], st[t][u][0][3], h1, l1);
          split2(st[t][u][1][0], st[t][u][1][1], h2, l2);
          split2(st[t][u][1][2], st[t][u][1][3], h3, l3);
          const uint4 sh = make_uint4(h0, h1, h2, h3), sl = make_uint4(l0, l1, l2, l3);
#pragma unroll
          for (int pt = 0; pt < PT; ++pt) {
            const uint4 b = cat2(gbop(u, pt, false), gbop(u, pt, true));
            f32x4& c = t == 0 ? acc0[pt] : acc1[pt];
            c = mfma_b32(sh, b, c);
            c = mfma_b32(sl, b, c);
          }
        } else {
          unsigned h0, l0, h1, l1;
          split2(st[t][u][0][0], st[t][u][0][1], h0, l0);
          split2(st[t][u][0][2], st[t][u][0][3], h1, l1);
          const uint2 sh = make_uint2(h0, h1), sl = make_uint2(l0, l1);
#pragma unroll
          for (int pt = 0; pt < PT; ++pt) {
            f32x4& c = t == 0 ? acc0[pt] : acc1[pt];
            const uint2 b = gbop(u, pt, false);
            c = mfma_b32h(sh, b, c);
            c = mfma_b32h(sl, b, c);
          }
        }
      }
    if (!more) break;
    // the next block's G_B rows: their latency is covered by its stage 1
    load_b(ni, nq);
    if (reload) take_a();
    i = ni;
    q = nq;
  }
}

// NA = 2 only where one mode index per trip takes few enough registers;
// otherwise the two a-tiles one after the other.  With na == 1 only acc0 is
// written.
template <int KC, int PT>
__device__ __forceinline__ void lds16_tiles_u(const StepOp& op, const TTC_LDS uint16_t* In, int lo, int na,
                                              const int (&at)[2], int s0, int S, f32x4 (&acc0)[SW_MAXT],
                                              f32x4 (&acc1)[SW_MAXT]) {
  constexpr int U = TripWidth16<KC, PT>::U;
  // (the rest of the 256 registers: offsets, masks, addresses, temporaries
  // and what the step keeps live around the call; a larger bound spilled in
  // the loop and measured slower on the 4096-pair batch)
  if constexpr (U == 1 && TripRegs<KC, PT, 2, 1>::n <= 160) {
    if (na == 2) {
      lds16_tiles<KC, PT, 2, 1>(op, In, lo, at, s0, S, acc0, acc1);
      return;
    }
  }
  lds16_tiles<KC, PT, 1, U>(op, In, lo, at, s0, S, acc0, acc0);
  if (na == 2) {
    const int a1[2] = {at[1], at[1]};
    lds16_tiles<KC, PT, 1, U>(op, In, lo, a1, s0, S, acc1, acc1);
  }
}

template <int KC>
__device__ __forceinline__ void lds16_tiles_p(const StepOp& op, const TTC_LDS uint16_t* In, int lo, int na,
                                              const int (&at)[2], int s0, int S, f32x4 (&acc0)[SW_MAXT],
                                              f32x4 (&acc1)[SW_MAXT]) {
  switch ((op.Nb + 15) >> 4) {
    case 1: lds16_tiles_u<KC, 1>(op, In, lo, na, at, s0, S, acc0, acc1); break;
    case 2: lds16_tiles_u<KC, 2>(op, In, lo, na, at, s0, S, acc0, acc1); break;
    case 3: lds16_tiles_u<KC, 3>(op, In, lo, na, at, s0, S, acc0, acc1); break;
    case 4: lds16_tiles_u<KC, 4>(op, In, lo, na, at, s0, S, acc0, acc1); break;
    case 5: lds16_tiles_u<KC, 5>(op, In, lo, na, at, s0, S, acc0, acc1); break;
    case 6: lds16_tiles_u<KC, 6>(op, In, lo, na, at, s0, S, acc0, acc1); break;
    case 7: lds16_tiles_u<KC, 7>(op, In, lo, na, at, s0, S, acc0, acc1); break;
    default: lds16_tiles_u<KC, 8>(op, In, lo, na, at, s0, S, acc0, acc1); break;
  }
}

// na a-tiles (1 or 2) of one wave: mode indices s0, s0 + S, ...
__device__ __forceinline__ void lds16_tiles_v(const StepOp& op, const TTC_LDS uint16_t* In, int lo, int na,
                                              const int (&at)[2], int s0, int S, f32x4 (&acc0)[SW_MAXT],
                                              f32x4 (&acc1)[SW_MAXT]) {
  switch ((op.Ka + 15) >> 4) {
    case 1: lds16_tiles_p<1>(op, In, lo, na, at, s0, S, acc0, acc1); break;
    case 2: lds16_tiles_p<2>(op, In, lo, na, at, s0, S, acc0, acc1); break;
    case 3: lds16_tiles_p<3>(op, In, lo, na, at, s0, S, acc0, acc1); break;
    case 4: lds16_tiles_p<4>(op, In, lo, na, at, s0, S, acc0, acc1); break;
    case 5: lds16_tiles_p<5>(op, In, lo, na, at, s0, S, acc0, acc1); break;
    case 6: lds16_tiles_p<6>(op, In, lo, na, at, s0, S, acc0, acc1); break;
    case 7: lds16_tiles_p<7>(op, In, lo, na, at, s0, S, acc0, acc1); break;
    default: lds16_tiles_p<8>(op, In, lo, na, at, s0, S, acc0, acc1); break;
  }
}

// Row pitch (BF16 elements) of the LDS stage that holds one 32-wide block
// of G_B: a byte stride of 16 x 5, so 16 lanes reading 16 bytes from 16
// consecutive rows touch disjoint banks.
constexpr int kStagePitch = 40;

__device__ __forceinline__ u32x4_t raw4_at(const CoreRes& c, int off) {
  return __builtin_amdgcn_raw_buffer_load_b128(c.r, off, 0, 0);
}

// The step of lds16_tiles for shapes where every wave walks all mode indices
// (no mode-index split) and G_B is wide: each trip's G_B block is loaded once
// by the whole workgroup instead of by every wave.  Thread t loads row t / 2
// of the block (sixteen b' from 16 (t % 2), with aligned 16-byte loads and a
// funnel shift), masks entries past Kb and writes them to the LDS stage in
// the order of the stage-2 operands (position 8g + j of a row holds the b'
// that lane group g puts in slot j); waves read their operands from there.
// A trip: stage 1 (In^T, G_A), the next G_A rows if a mode index ends,
// barrier (the stage is free), stage write, loads of the next block,
// barrier (the stage is full), stage 2.  Every wave of the workgroup calls
// this with the same step (na = 0, 1 or 2 output row tiles of its own), so
// the barriers match.
template <int KC, int PT, int NT>
__device__ __forceinline__ void lds16_tiles_staged(const StepOp& op, const TTC_LDS uint16_t* __restrict__ In, int lo,
                                                   TTC_LDS uint16_t* __restrict__ stage, int na, const int (&at)[2],
                                                   f32x4 (&acc0)[SW_MAXT], f32x4 (&acc1)[SW_MAXT]) {
  static_assert(NT >= 2 * 16 * PT, "one staging thread per half row");
  constexpr int KP = KC / 2, KT = KC & 1, KPA = KP > 0 ? KP : 1;
  const int lane = threadIdx.x & 63, li = lane & 15, g = lane >> 4;
  const int I = __builtin_amdgcn_readfirstlane(op.I), Ka = __builtin_amdgcn_readfirstlane(op.Ka),
            Kb = __builtin_amdgcn_readfirstlane(op.Kb);
  const int QT = (Kb + 15) >> 4, QB = (QT + 1) >> 1;
  const int ip = lds16_pitch(Ka);
  const long ta = (long)op.Ma * I * Ka, tb = (long)op.Nb * I * Kb;
  int aal[2];
#pragma unroll
  for (int t = 0; t < 2; ++t) aal[t] = ((at[t] * 16 + li) * I * Ka * 2) & ~3;
  const int apar = ((li * I * Ka) & 1) << 1;
  const bool apart = (Ka & 15) != 0;
  const uint2 ma0 = KT ? keep4(32 * KP + 4 * g, Ka) : keep4(32 * (KP - 1) + 8 * g, Ka);
  const uint2 ma1 = keep4(32 * (KP - 1) + 8 * g + 4, Ka);
  // staging: row sr of the block, elements 16 sh2 .. 16 sh2 + 15
  const int sr = threadIdx.x >> 1, sh2 = threadIdx.x & 1;
  const bool srow = sr < 16 * PT;
  const int srel = (sr * I * Kb + 16 * sh2) * 2;
  const int sal = srel & ~3, spar = srel & 2;

  uint4 ga[2][KPA];
  uint2 gat[2];
  u32x3 gar[2][KPA][2], gatr[2];
  int sha = 0;
  u32x4_t sr0, sr1;
  unsigned sr2 = 0;
  int shs = 0;

  auto load_a = [&](int i0) {
    const CoreRes ra = core_rsrc(op.ga, (long)i0 * Ka, ta, 2);
    const int corr = (apar & ra.adj) << 1;
    sha = (apar ^ ra.adj) << 3;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      if (t >= na) break;
      const int o = aal[t] + corr;
#pragma unroll
      for (int c = 0; c < KP; ++c) {
        gar[t][c][0] = raw_at(ra, o + (32 * c + 8 * g) * 2);
        gar[t][c][1] = raw_at(ra, o + (32 * c + 8 * g + 4) * 2);
      }
      if constexpr (KT) gatr[t] = raw_at(ra, o + (32 * KP + 4 * g) * 2);
    }
  };
  auto take_a = [&]() {
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      if (t >= na) break;
#pragma unroll
      for (int c = 0; c < KP; ++c) ga[t][c] = cat2(take_raw(gar[t][c][0], sha), take_raw(gar[t][c][1], sha));
      if constexpr (KT) gat[t] = take_raw(gatr[t], sha);
      if (apart) {
        if constexpr (KT) {
          gat[t] = and2(gat[t], ma0);
        } else {
          uint4& v = ga[t][KP - 1];
          v = make_uint4(v.x & ma0.x, v.y & ma0.y, v.z & ma1.x, v.w & ma1.y);
        }
      }
    }
  };
  // raw loads of this thread's part of block q of mode index i0
  auto load_s = [&](int i0, int q) {
    if (!srow) return;
    const CoreRes rb = core_rsrc(op.gb, (long)i0 * Kb + 32 * q, tb, 2);
    const int o = sal + ((spar & rb.adj) << 1);
    shs = (spar ^ rb.adj) << 3;
    sr0 = raw4_at(rb, o);
    sr1 = raw4_at(rb, o + 16);
    sr2 = __builtin_amdgcn_raw_buffer_load_b32(rb.r, o + 32, 0, 0);
  };
  // the loaded part of block q, masked past Kb, into the stage
  auto write_s = [&](int q) {
    if (!srow) return;
    const unsigned w[9] = {sr0[0], sr0[1], sr0[2], sr0[3], sr1[0], sr1[1], sr1[2], sr1[3], sr2};
    const int e0 = 32 * q + 16 * sh2;
    TTC_LDS uint16_t* row = stage + sr * kStagePitch;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      uint2 v = make_uint2(__builtin_amdgcn_alignbit(w[2 * m + 1], w[2 * m], shs),
                           __builtin_amdgcn_alignbit(w[2 * m + 2], w[2 * m + 1], shs));
      if (e0 + 4 * m + 4 > Kb) v = and2(v, keep4(e0 + 4 * m, Kb));
      const int hh = 4 * sh2 + m;
      const int pos = hh < 4 ? 8 * hh : 8 * (hh - 4) + 4;
      *reinterpret_cast<TTC_LDS uint2*>(row + pos) = v;
    }
  };

  load_a(0);
  load_s(0, 0);
  take_a();
  int i = 0, q = 0;
  for (;;) {
    int ni = i, nq = q + 1;
    if (nq == QB) {
      nq = 0;
      ni = i + 1;
    }
    const bool more = ni < I;
    const bool full = 2 * q + 1 < QT;
    // stage 1: S^T rows b' = 32q + 16h + (0..15) of each of the wave's tiles
    f32x4 st[2][2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (h == 1 && !full) break;
      const TTC_LDS uint16_t* row = In + (32 * q + 16 * h + li) * ip;
#pragma unroll
      for (int t = 0; t < 2; ++t) st[t][h] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int c = 0; c < KP; ++c) {
        const uint4 vh = *reinterpret_cast<const TTC_LDS uint4*>(row + 32 * c + 8 * g);
        const uint4 vl = *reinterpret_cast<const TTC_LDS uint4*>(row + lo + 32 * c + 8 * g);
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          if (t >= na) break;
          st[t][h] = mfma_b32(vh, ga[t][c], st[t][h]);
          st[t][h] = mfma_b32(vl, ga[t][c], st[t][h]);
        }
      }
      if constexpr (KT) {
        const uint2 vh = *reinterpret_cast<const TTC_LDS uint2*>(row + 32 * KP + 4 * g);
        const uint2 vl = *reinterpret_cast<const TTC_LDS uint2*>(row + lo + 32 * KP + 4 * g);
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          if (t >= na) break;
          st[t][h] = mfma_b32h(vh, gat[t], st[t][h]);
          st[t][h] = mfma_b32h(vl, gat[t], st[t][h]);
        }
      }
    }
    const bool reload = more && nq == 0;
    if (reload) load_a(ni);
    __syncthreads();  // every wave is done with the stage's previous block
    write_s(q);
    if (more) load_s(ni, nq);
    __syncthreads();  // the stage holds block q
    // stage 2 with the G_B operands from the stage
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      if (t >= na) break;
      if (full) {
        unsigned h0, l0, h1, l1, h2, l2, h3, l3;
        split2(st[t][0][0], st[t][0][1], h0, l0);
        split2(st[t][0][2], st[t][0][3], h1, l1);
        split2(st[t][1][0], st[t][1][1], h2, l2);
        split2(st[t][1][2], st[t][1][3], h3, l3);
        const uint4 sh = make_uint4(h0, h1, h2, h3), sl = make_uint4(l0, l1, l2, l3);
#pragma unroll
        for (int pt = 0; pt < PT; ++pt) {
          const uint4 b = *reinterpret_cast<const TTC_LDS uint4*>(stage + (pt * 16 + li) * kStagePitch + 8 * g);
          f32x4& c = t == 0 ? acc0[pt] : acc1[pt];
          c = mfma_b32(sh, b, c);
          c = mfma_b32(sl, b, c);
        }
      } else {
        unsigned h0, l0, h1, l1;
        split2(st[t][0][0], st[t][0][1], h0, l0);
        split2(st[t][0][2], st[t][0][3], h1, l1);
        const uint2 sh = make_uint2(h0, h1), sl = make_uint2(l0, l1);
#pragma unroll
        for (int pt = 0; pt < PT; ++pt) {
          const uint2 b = *reinterpret_cast<const TTC_LDS uint2*>(stage + (pt * 16 + li) * kStagePitch + 8 * g);
          f32x4& c = t == 0 ? acc0[pt] : acc1[pt];
          c = mfma_b32h(sh, b, c);
          c = mfma_b32h(sl, b, c);
        }
      }
    }
    if (!more) break;
    if (reload) take_a();
    i = ni;
    q = nq;
  }
}

// VGPRs of a staged trip: both output tiles, the G_A operands and their raw
// reload (live together: the operands carry over to the next block), the
// stage-1 tiles, the staging thread's raw dwords.
template <int KC, int PT>
struct StagedRegs {
  static constexpr int KP = KC / 2, KT = KC & 1;
  static constexpr int n = 2 * PT * 4 + 2 * (KP * 4 + KT * 2) + 2 * (KP * 6 + KT * 3) + 16 + 9;
};

template <int KC, int PT, int NT>
__device__ __forceinline__ void lds16_staged_t(const StepOp& op, const TTC_LDS uint16_t* In, int lo,
                                               TTC_LDS uint16_t* stage, int na, const int (&at)[2],
                                               f32x4 (&acc0)[SW_MAXT], f32x4 (&acc1)[SW_MAXT]) {
  // larger staged shapes spilled and measured slower on the 4096-pair batch
  if constexpr (StagedRegs<KC, PT>::n <= 160) {
    lds16_tiles_staged<KC, PT, NT>(op, In, lo, stage, na, at, acc0, acc1);
  } else {
    // too many registers for a staged trip: each wave streams its own G_B
    if (na > 0) lds16_tiles_u<KC, PT>(op, In, lo, na, at, 0, 1, acc0, acc1);
  }
}

template <int KC, int NT>
__device__ __forceinline__ void lds16_staged_p(const StepOp& op, const TTC_LDS uint16_t* In, int lo,
                                               TTC_LDS uint16_t* stage, int na, const int (&at)[2],
                                               f32x4 (&acc0)[SW_MAXT], f32x4 (&acc1)[SW_MAXT]) {
  switch ((op.Nb + 15) >> 4) {
    case 3: lds16_staged_t<KC, 3, NT>(op, In, lo, stage, na, at, acc0, acc1); break;
    case 4: lds16_staged_t<KC, 4, NT>(op, In, lo, stage, na, at, acc0, acc1); break;
    case 5: lds16_staged_t<KC, 5, NT>(op, In, lo, stage, na, at, acc0, acc1); break;
    case 6: lds16_staged_t<KC, 6, NT>(op, In, lo, stage, na, at, acc0, acc1); break;
    case 7: lds16_staged_t<KC, 7, NT>(op, In, lo, stage, na, at, acc0, acc1); break;
    default: lds16_staged_t<KC, 8, NT>(op, In, lo, stage, na, at, acc0, acc1); break;
  }
}

// The staged step for pad16(Nb) >= 48 (na output row tiles of this wave).
template <int NT>
__device__ __forceinline__ void lds16_staged_v(const StepOp& op, const TTC_LDS uint16_t* In, int lo,
                                               TTC_LDS uint16_t* stage, int na, const int (&at)[2],
                                               f32x4 (&acc0)[SW_MAXT], f32x4 (&acc1)[SW_MAXT]) {
  switch ((op.Ka + 15) >> 4) {
    case 1: lds16_staged_p<1, NT>(op, In, lo, stage, na, at, acc0, acc1); break;
    case 2: lds16_staged_p<2, NT>(op, In, lo, stage, na, at, acc0, acc1); break;
    case 3: lds16_staged_p<3, NT>(op, In, lo, stage, na, at, acc0, acc1); break;
    case 4: lds16_staged_p<4, NT>(op, In, lo, stage, na, at, acc0, acc1); break;
    case 5: lds16_staged_p<5, NT>(op, In, lo, stage, na, at, acc0, acc1); break;
    case 6: lds16_staged_p<6, NT>(op, In, lo, stage, na, at, acc0, acc1); break;
    case 7: lds16_staged_p<7, NT>(op, In, lo, stage, na, at, acc0, acc1); break;
    default: lds16_staged_p<8, NT>(op, In, lo, stage, na, at, acc0, acc1); break;
  }
}

// Store (FIRST) or add the a-tile `at` of Out into the two planes: acc[pt][v]
// is Out[at*16 + 4g + v, pt*16 + li].  native: Out^T layout (rows b, pitch
// lds16_pitch(Ma)), one 8-byte write per plane and tile; else Out layout
// (rows a, pitch lds16_pitch(Nb)).  Entries outside Ma x Nb are written as
// zeros.  Adding reads the old hi + lo, adds in FP32 and splits again.
template <bool FIRST>
__device__ __forceinline__ void lds16_put(TTC_LDS uint16_t* Out, int lo, bool native, int Ma, int Nb, int at,
                                          const f32x4 (&acc)[SW_MAXT]) {
  const int lane = threadIdx.x & 63, li = lane & 15, g = lane >> 4;
  const int PT = (Nb + 15) >> 4;
  const int a0 = at * 16 + 4 * g;
#pragma unroll
  for (int pt = 0; pt < SW_MAXT; ++pt) {
    if (pt >= PT) break;
    const int b = pt * 16 + li;
    f32x4 v;
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = (a0 + u < Ma && b < Nb) ? acc[pt][u] : 0.f;
    if (native) {
      TTC_LDS uint2* ph = reinterpret_cast<TTC_LDS uint2*>(Out + b * lds16_pitch(Ma) + a0);
      TTC_LDS uint2* pl = reinterpret_cast<TTC_LDS uint2*>(Out + lo + b * lds16_pitch(Ma) + a0);
      if (!FIRST) {
        const uint2 oh = *ph, ol = *pl;
        v[0] += bf16_lo(oh.x) + bf16_lo(ol.x);
        v[1] += bf16_hi(oh.x) + bf16_hi(ol.x);
        v[2] += bf16_lo(oh.y) + bf16_lo(ol.y);
        v[3] += bf16_hi(oh.y) + bf16_hi(ol.y);
      }
      uint2 h, l;
      split2(v[0], v[1], h.x, l.x);
      split2(v[2], v[3], h.y, l.y);
      *ph = h;
      *pl = l;
    } else {
      const int np = lds16_pitch(Nb);
      if (!FIRST) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int e = (a0 + u) * np + b;
          v[u] += bf16_to_f32(Out[e]) + bf16_to_f32(Out[lo + e]);
        }
      }
      unsigned h01, l01, h23, l23;
      split2(v[0], v[1], h01, l01);
      split2(v[2], v[3], h23, l23);
      const unsigned hh[2] = {h01, h23}, ll[2] = {l01, l23};
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = (a0 + u) * np + b;
        Out[e] = (uint16_t)(hh[u >> 1] >> (16 * (u & 1)));
        Out[lo + e] = (uint16_t)(ll[u >> 1] >> (16 * (u & 1)));
      }
    }
  }
}

// The in-place step (see lds_step_inplace) on the BF16 planes: each wave
// keeps at most two output tiles in registers until every wave has read In,
// then the tiles overwrite it in the fixed order of their mode-index parts.
// `stage` (kStagePitch x 128 BF16, or null) lets steps with wide G_B and no
// mode-index split stage G_B in LDS.  Ends with a workgroup barrier.
template <int NW>
__device__ __forceinline__ void lds16_step_inplace(const StepOp& op, TTC_LDS uint16_t* Buf, int lo, bool native,
                                                   TTC_LDS uint16_t* stage) {
  const int RT = (op.Ma + 15) >> 4;  // <= 8 <= 2 NW
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  int S = 1, best = ((RT + NW - 1) / NW) * op.I;
  for (int c = 2; c <= 2 * NW && c <= op.I && RT * c <= 2 * NW; c *= 2) {
    const int cost = ((RT * c + NW - 1) / NW) * ((op.I + c - 1) / c);
    if (cost < best) {
      best = cost;
      S = c;
    }
  }
  const int items = RT * S;
  const int item0 = w, item1 = w + NW;
  f32x4 keep[SW_MAXT], acc[SW_MAXT];
#pragma unroll
  for (int t = 0; t < SW_MAXT; ++t) keep[t] = acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  if (S == 1 && stage && op.Nb > 32) {
    // wide G_B, every wave on all mode indices: the workgroup stages G_B
    const int na = (item0 < items) + (item1 < items);
    const int at[2] = {item0, item1};
    lds16_staged_v<NW * 64>(op, Buf, lo, stage, na, at, keep, acc);
  } else if (S == 1 && item1 < items) {
    // both of the wave's a-tiles, every mode index
    const int at[2] = {item0, item1};
    lds16_tiles_v(op, Buf, lo, 2, at, 0, 1, keep, acc);
  } else {
    // one (a-tile, mode-index part) item per pass
#pragma unroll 1
    for (int it = 0; it < 2; ++it) {
      const int item = w + it * NW;
#pragma unroll
      for (int t = 0; t < SW_MAXT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
      if (item < items) {
        const int at[2] = {item % RT, item % RT};
        lds16_tiles_v(op, Buf, lo, 1, at, item / RT, S, acc, acc);
      }
      if (it == 0) {
#pragma unroll
        for (int t = 0; t < SW_MAXT; ++t) keep[t] = acc[t];
      }
    }
  }
  __syncthreads();  // In fully read
  for (int ss = 0; ss < S; ++ss) {
    if (item0 < items && item0 / RT == ss) {
      if (ss == 0) lds16_put<true>(Buf, lo, native, op.Ma, op.Nb, item0 % RT, keep);
      else lds16_put<false>(Buf, lo, native, op.Ma, op.Nb, item0 % RT, keep);
    }
    if (item1 < items && item1 / RT == ss) {
      if (ss == 0) lds16_put<true>(Buf, lo, native, op.Ma, op.Nb, item1 % RT, acc);
      else lds16_put<false>(Buf, lo, native, op.Ma, op.Nb, item1 % RT, acc);
    }
    __syncthreads();
  }
}

// Value of element e of an interface held as BF16 planes.
__device__ __forceinline__ float lds16_get(const TTC_LDS uint16_t* V, int lo, int e) {
  return bf16_to_f32(V[e]) + bf16_to_f32(V[lo + e]);
}

// Per-thread part of <X, Y> (see lds_final_k) with V_1 held as BF16 planes
// (rows p', pitch lds16_pitch(R1)); the product with G_x^(0) on FP32 MFMA,
// the sum with G_y^(0) in FP64.
template <int KC, int NW>
__device__ __forceinline__ double lds16_final_k(const void* gx0, const void* gy0, int I, int R1, int P1,
                                                const TTC_LDS uint16_t* V, int lo) {
  typedef Raw4<bf16_t> R4;
  const int lane = threadIdx.x & 63, li = lane & 15, g = lane >> 4;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int MT = (I + 15) >> 4, NTl = (P1 + 15) >> 4, vp = lds16_pitch(R1);
  const CoreRes rx = core_rsrc(gx0, 0, (long)I * R1, 2);
  const TTC_GLOBAL bf16_t* gy = gptr<bf16_t>(gy0);
  double s = 0.0;
  for (int item = w; item < MT * NTl; item += NW) {
    const int mt = item % MT, nt = item / MT;
    const int xoff = ((mt * 16 + li) * R1 + 4 * g) * 2;
    const int vrow = (nt * 16 + li) * vp + 4 * g;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kc = 0; kc < KC; ++kc) {
      const uint2 a = R4::load(rx, xoff + kc * 16 * 2);
      const uint2 bh = *reinterpret_cast<const TTC_LDS uint2*>(V + vrow + kc * 16);
      const uint2 bl = *reinterpret_cast<const TTC_LDS uint2*>(V + lo + vrow + kc * 16);
      const float b[4] = {bf16_lo(bh.x) + bf16_lo(bl.x), bf16_hi(bh.x) + bf16_hi(bl.x), bf16_lo(bh.y) + bf16_lo(bl.y),
                          bf16_hi(bh.y) + bf16_hi(bl.y)};
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const float av = (kc * 16 + 4 * g + u < R1) ? R4::get(a, u) : 0.f;
        acc = mfma4(av, b[u], acc);
      }
    }
    const int p = nt * 16 + li;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = mt * 16 + 4 * g + v;
      if (i < I && p < P1) s += (double)acc[v] * (double)cvt<float>(gy[i * P1 + p]);
    }
  }
  return s;
}

template <int NW>
__device__ __forceinline__ double lds16_final(const void* gx0, const void* gy0, int I, int R1, int P1,
                                              const TTC_LDS uint16_t* V, int lo) {
  switch ((R1 + 15) >> 4) {
    case 1: return lds16_final_k<1, NW>(gx0, gy0, I, R1, P1, V, lo);
    case 2: return lds16_final_k<2, NW>(gx0, gy0, I, R1, P1, V, lo);
    case 3: return lds16_final_k<3, NW>(gx0, gy0, I, R1, P1, V, lo);
    case 4: return lds16_final_k<4, NW>(gx0, gy0, I, R1, P1, V, lo);
    case 5: return lds16_final_k<5, NW>(gx0, gy0, I, R1, P1, V, lo);
    case 6: return lds16_final_k<6, NW>(gx0, gy0, I, R1, P1, V, lo);
    case 7: return lds16_final_k<7, NW>(gx0, gy0, I, R1, P1, V, lo);
    default: return lds16_final_k<8, NW>(gx0, gy0, I, R1, P1, V, lo);
  }
}

}  // namespace ttc
