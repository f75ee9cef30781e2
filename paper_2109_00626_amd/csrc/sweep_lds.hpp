// Interface sweep step with both interfaces resident in LDS, zero-padded.
//
// One right-to-left step on core k computes
//   Out[a, b] = sum_i sum_{a', b'} G_A[a, i, a'] In[a', b'] G_B[b, i, b']
// where (A, B) = (X, Y) gives V_k = sum_i G_x[:, i, :] V_{k+1} G_y[:, i, :]^T
// ("x first") and (A, B) = (Y, X) gives its transpose ("y first").  The
// two orders cost different FLOPs when the X and Y ranks differ; each step
// takes the cheaper one for its padded tile counts.
//
// Per mode index i the step is two chained MFMA products (see
// sweep_steps.hpp for the accumulator-as-operand argument):
//   S_i^T (Kb x Ma) = In^T . G_A[:, i, :]^T      (K = Ka)
//   Out   (Ma x Nb) += S_i . G_B[:, i, :]^T        (K = Kb)
// Interfaces are stored in LDS as In^T (rows b', columns a'), with every
// dimension padded to a multiple of 16 with zeros, so the operand reads are
// 16-byte LDS loads with no bounds logic, and a row pitch of 4 x (odd) floats
// so that 16 lanes reading 16 bytes from 16 consecutive rows touch disjoint
// banks.  A step writes its output in the orientation the next step reads
// (its own transposed layout when the next step has the same order, else
// the plain layout), with zeros outside the valid block.
//
// Core elements stream from global memory straight into registers, four
// consecutive elements of a core row per lane in one vector load; each core
// element is read once per workgroup.  The loads of the next (i, column-slice)
// iteration are issued before the MFMAs of the current one.
#pragma once
#include "sweep_steps.hpp"

namespace ttc {

__host__ __device__ __forceinline__ int pad16(int n) { return (n + 15) & ~15; }
// Row pitch (floats) of an LDS interface whose rows hold n valid entries.
__host__ __device__ __forceinline__ int lds_pitch(int n) { return pad16(n) + 4; }

// True when the "y first" order needs fewer padded MFMA tiles than "x first"
// for the step on a core with X ranks (Rp, Rn) and Y ranks (Pp, Pn).
__host__ __device__ __forceinline__ bool step_y_first(int Rp, int Rn, int Pp, int Pn) {
  const long cx = (long)pad16(Rp) * pad16(Pn) * (pad16(Rn) + pad16(Pp));
  const long cy = (long)pad16(Pp) * pad16(Rn) * (pad16(Pn) + pad16(Rp));
  return cy < cx;
}

// Floats of one LDS interface buffer able to hold R x P in either layout.
__host__ __device__ __forceinline__ int lds_iface_elems(int R, int P) {
  const int t = pad16(P) * lds_pitch(R), n = pad16(R) * lds_pitch(P);
  return t > n ? t : n;
}

// One step's operands: G_A is [Ma][I][Ka], G_B is [Nb][I][Kb] (row-major).
struct StepOp {
  const void* ga;
  const void* gb;
  int Ma, Ka, Nb, Kb, I;
};

// Core reads go through raw buffer loads: the resource spans one core, so
// lanes whose offset falls past its end read zeros instead of faulting, and
// no row or address needs clamping.  Each resource starts at the first
// element of the current (mode index, column slice), which keeps the
// per-lane byte offsets constant over the whole step.  Buffer loads of more
// than one word need word-aligned addresses, so a resource starts at the
// word holding its first element and `adj` (0 or 2 bytes) is added to every
// offset; its size is rounded up to whole words (the last word of a core
// shares a page with the core's last element, so it is always mapped).
struct CoreRes {
  __amdgpu_buffer_rsrc_t r;
  int adj;
};
__device__ __forceinline__ CoreRes core_rsrc(const void* base, long first, long total, int esz) {
  // first, total: elements; the resource covers [first, total).  The
  // arguments are uniform; readfirstlane lets the compiler keep the
  // resource in scalar registers.
  const uintptr_t a = reinterpret_cast<uintptr_t>(base) + (uintptr_t)(first * esz);
  const uintptr_t a4 = a & ~(uintptr_t)3;
  const int adj = (int)(a - a4);
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)a4);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(a4 >> 32));
  const int bytes = __builtin_amdgcn_readfirstlane((int)((adj + (total - first) * esz + 3) & ~3L));
  char* p = reinterpret_cast<char*>(((uintptr_t)hi << 32) | lo);
  CoreRes c;
  c.r = __builtin_amdgcn_make_buffer_rsrc(p, (short)0, bytes, 0x00020000);
  c.adj = __builtin_amdgcn_readfirstlane(adj);
  return c;
}

// Four consecutive core elements at byte offset `off` of the resource, as
// raw bits (FP32: four words; BF16: two words of two elements each).
template <typename Tin>
struct Raw4;
template <>
struct Raw4<float> {
  typedef f32x4 type;
  // FP32 cores are word-aligned, so adj is 0
  __device__ __forceinline__ static f32x4 load(const CoreRes& c, int off) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b128(c.r, off, 0, 0);
    return f32x4{__uint_as_float(v[0]), __uint_as_float(v[1]), __uint_as_float(v[2]), __uint_as_float(v[3])};
  }
  __device__ __forceinline__ static float get(const f32x4& v, int u) { return v[u]; }
  // as FP32, elements u with keep[u] false set to zero
  __device__ __forceinline__ static f32x4 to_f32(const f32x4& v, const bool keep[4]) {
    return f32x4{keep[0] ? v[0] : 0.f, keep[1] ? v[1] : 0.f, keep[2] ? v[2] : 0.f, keep[3] ? v[3] : 0.f};
  }
  __device__ __forceinline__ static f32x4 to_f32(const f32x4& v) { return v; }
};
template <>
struct Raw4<bf16_t> {
  typedef uint2 type;
  // the four elements lie in three words starting at the word-aligned byte
  // offset below; a funnel shift by 0 or 16 bits extracts them
  __device__ __forceinline__ static uint2 load(const CoreRes& c, int off) {
    const int e = off + c.adj;
    const auto v = __builtin_amdgcn_raw_buffer_load_b96(c.r, e & ~3, 0, 0);
    const unsigned sh = (unsigned)(e & 2) << 3;
    return make_uint2(__builtin_amdgcn_alignbit(v[1], v[0], sh), __builtin_amdgcn_alignbit(v[2], v[1], sh));
  }
  __device__ __forceinline__ static float get(const uint2& v, int u) {
    const unsigned w = (u < 2) ? v.x : v.y;
    return __uint_as_float((u & 1) ? (w & 0xFFFF0000u) : (w << 16));
  }
  __device__ __forceinline__ static f32x4 to_f32(const uint2& v, const bool keep[4]) {
    return f32x4{keep[0] ? get(v, 0) : 0.f, keep[1] ? get(v, 1) : 0.f, keep[2] ? get(v, 2) : 0.f,
                 keep[3] ? get(v, 3) : 0.f};
  }
  __device__ __forceinline__ static f32x4 to_f32(const uint2& v) {
    return f32x4{get(v, 0), get(v, 1), get(v, 2), get(v, 3)};
  }
};

// s_waitcnt immediate for "vector memory count 0" (gfx9 encoding: expcnt
// and lgkmcnt fields at their no-wait maxima).
constexpr int kWaitVmcnt0 = (0x7 << 4) | (0xF << 8);

__device__ __forceinline__ f32x4 mfma4(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Resource over elements [first, total) of a core when `valid`, else of zero
// bytes (every load reads zero).  Branch-free, so that the resource stays in
// scalar registers.
__device__ __forceinline__ CoreRes core_rsrc_if(bool valid, const void* base, long first, long total, int esz) {
  const uintptr_t a = reinterpret_cast<uintptr_t>(base) + (uintptr_t)(first * esz);
  const uintptr_t a4 = a & ~(uintptr_t)3;
  const int adj = (int)(a - a4);
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)a4);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(a4 >> 32));
  const long span = (adj + (total - first) * esz + 3) & ~3L;
  const int bytes = __builtin_amdgcn_readfirstlane(valid ? (int)span : 0);
  char* p = reinterpret_cast<char*>(((uintptr_t)hi << 32) | lo);
  CoreRes c;
  c.r = __builtin_amdgcn_make_buffer_rsrc(p, (short)0, bytes, 0x00020000);
  c.adj = __builtin_amdgcn_readfirstlane(adj);
  return c;
}

// Mode indices a wave handles per loop trip for the tile counts KC, PT: small
// tiles take several, so that each trip's MFMA work covers the latency of
// the next trip's loads (issued at the trip's start and waited for at its
// end), within the register budget of the largest tiles.
template <int KC, int PT>
struct TripWidth {
  static constexpr int U = (KC + PT <= 4) ? 4 : (KC + PT <= 8) ? 2 : 1;
};

// Accumulate mode indices i = s0, s0 + S, ... into the a-tile `at` of Out
// (its PT b-tiles, in acc).  KC = pad16(Ka) / 16, PT = pad16(Nb) / 16.
// Values of core rows past Ka (resp. Kb) are the next entries of the core;
// they meet zero padding of In, and are also masked to zero so that only
// the operation's own elements reach the sums.  A loop trip covers U mode
// indices i, i + S, ..., i + (U - 1) S (those past the core read zeros) and
// one 16-wide slice qt of b'; the U stage-1 products share one read of the
// In^T slice and form independent MFMA chains.  An index past I gets an
// empty resource (its start may still lie inside the core, in another row).
template <typename Tin, int KC, int PT>
__device__ __forceinline__ void lds_tile(const StepOp& op, const TTC_LDS float* __restrict__ In, int at, int s0, int S,
                                         f32x4 (&acc)[SW_MAXT]) {
  typedef Raw4<Tin> R4;
  typedef typename R4::type raw_t;
  constexpr int esz = sizeof(Tin);
  constexpr int U = TripWidth<KC, PT>::U;
  const int lane = threadIdx.x & 63, li = lane & 15, g = lane >> 4;
  // the step's shape is the same in every lane (scalar registers, scalar branches)
  const int I = __builtin_amdgcn_readfirstlane(op.I), Ka = __builtin_amdgcn_readfirstlane(op.Ka),
            Kb = __builtin_amdgcn_readfirstlane(op.Kb);
  const int QT = (Kb + 15) >> 4;
  const int ip = lds_pitch(Ka);
  const long ta = (long)op.Ma * I * Ka, tb = (long)op.Nb * I * Kb;
  // per-lane byte offsets: row start + 4g (+ 16 kc) elements
  const int aoff = ((at * 16 + li) * I * Ka + 4 * g) * esz;
  int boff[PT];
#pragma unroll
  for (int pt = 0; pt < PT; ++pt) boff[pt] = ((pt * 16 + li) * I * Kb + 4 * g) * esz;
  // masks of the last (partial) chunk along a' and of the last slice along b'
  bool ma[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) ma[u] = (KC - 1) * 16 + 4 * g + u < Ka;
  const TTC_LDS float* inl = In + li * ip + 4 * g;
  if (s0 >= I) return;
  const int step = U * S;
  const bool afull = (Ka & 15) == 0;  // no partial chunk along a

  // current operands as FP32 (masked), next ones as loaded
  f32x4 bx[U][KC], gv[U][PT];
  raw_t bxn[U][KC], gvn[U][PT];
  {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const CoreRes ra = core_rsrc_if(s0 + u * S < I, op.ga, (long)(s0 + u * S) * Ka, ta, esz);
      const CoreRes rb = core_rsrc_if(s0 + u * S < I, op.gb, (long)(s0 + u * S) * Kb, tb, esz);
#pragma unroll
      for (int kc = 0; kc < KC; ++kc) bxn[u][kc] = R4::load(ra, aoff + kc * 16 * esz);
#pragma unroll
      for (int pt = 0; pt < PT; ++pt) gvn[u][pt] = R4::load(rb, boff[pt]);
    }
    bool mb[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) mb[v] = 4 * g + v < Kb;
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int kc = 0; kc < KC - 1; ++kc) bx[u][kc] = R4::to_f32(bxn[u][kc]);
      bx[u][KC - 1] = R4::to_f32(bxn[u][KC - 1], ma);
#pragma unroll
      for (int pt = 0; pt < PT; ++pt) gv[u][pt] = R4::to_f32(gvn[u][pt], mb);
    }
    // all prologue loads done here, so no load issued before the loop is
    // still counted as pending inside it
    __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
  }
  int i = s0, qt = 0;
  for (;;) {
    int ni = i, nq = qt + 1;
    if (nq == QT) {
      nq = 0;
      ni = i + step;
    }
    const bool more = ni < I;
    if (more) {
      if (nq == 0) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const CoreRes ra = core_rsrc_if(ni + u * S < I, op.ga, (long)(ni + u * S) * Ka, ta, esz);
#pragma unroll
          for (int kc = 0; kc < KC; ++kc) bxn[u][kc] = R4::load(ra, aoff + kc * 16 * esz);
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const CoreRes rb = core_rsrc_if(ni + u * S < I, op.gb, (long)(ni + u * S) * Kb + nq * 16, tb, esz);
#pragma unroll
        for (int pt = 0; pt < PT; ++pt) gvn[u][pt] = R4::load(rb, boff[pt]);
      }
    }
    // S_i^T rows qt*16.. (b') from In^T rows and the lane's G_A row
    f32x4 av[KC];
#pragma unroll
    for (int kc = 0; kc < KC; ++kc) av[kc] = *reinterpret_cast<const TTC_LDS f32x4*>(inl + qt * 16 * ip + kc * 16);
    f32x4 st[U];
#pragma unroll
    for (int u = 0; u < U; ++u) st[u] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kc = 0; kc < KC; ++kc)
#pragma unroll
      for (int w = 0; w < 4; ++w)
#pragma unroll
        for (int u = 0; u < U; ++u) st[u] = mfma4(av[kc][w], bx[u][kc][w], st[u]);
    // Out[a-tile, b-tile pt] += S_i[:, qt-slice] . G_B[b-tile, i, qt-slice]^T
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int pt = 0; pt < PT; ++pt)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[pt] = mfma4(st[u][v], gv[u][pt][v], acc[pt]);

    if (!more) break;
    // the prefetched operands become current, masked past the row ends
    // (only a last, partial 16-wide slice or chunk has such entries)
    if (nq * 16 + 16 <= Kb) {
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int pt = 0; pt < PT; ++pt) gv[u][pt] = R4::to_f32(gvn[u][pt]);
    } else {
      bool mb[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) mb[v] = nq * 16 + 4 * g + v < Kb;
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int pt = 0; pt < PT; ++pt) gv[u][pt] = R4::to_f32(gvn[u][pt], mb);
    }
    if (nq == 0) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
#pragma unroll
        for (int kc = 0; kc < KC - 1; ++kc) bx[u][kc] = R4::to_f32(bxn[u][kc]);
        bx[u][KC - 1] = afull ? R4::to_f32(bxn[u][KC - 1]) : R4::to_f32(bxn[u][KC - 1], ma);
      }
    }
    i = ni;
    qt = nq;
  }
}

// Two a-tiles of one wave in one pass (all mode indices, S = 1), for shapes
// that take one mode index per trip: the In^T reads and the G_B operands are
// shared by the tiles, so a trip carries twice the MFMA work per load.  The
// G_A rows of both tiles are reloaded once per mode index, right after the
// last slice's stage-1 products have consumed them (their latency is covered
// by that slice's stage 2).
template <typename Tin, int KC, int PT>
__device__ __forceinline__ void lds_tile2(const StepOp& op, const TTC_LDS float* __restrict__ In, int at0, int at1,
                                          f32x4 (&acc0)[SW_MAXT], f32x4 (&acc1)[SW_MAXT]) {
  typedef Raw4<Tin> R4;
  typedef typename R4::type raw_t;
  constexpr int esz = sizeof(Tin);
  // FP32 loads land in the operand registers themselves (no raw copy)
  constexpr bool kDirect = sizeof(raw_t) == sizeof(f32x4);
  const int lane = threadIdx.x & 63, li = lane & 15, g = lane >> 4;
  const int I = __builtin_amdgcn_readfirstlane(op.I), Ka = __builtin_amdgcn_readfirstlane(op.Ka),
            Kb = __builtin_amdgcn_readfirstlane(op.Kb);
  const int QT = (Kb + 15) >> 4;
  const int ip = lds_pitch(Ka);
  const long ta = (long)op.Ma * I * Ka, tb = (long)op.Nb * I * Kb;
  const int aoff0 = ((at0 * 16 + li) * I * Ka + 4 * g) * esz;
  const int aoff1 = ((at1 * 16 + li) * I * Ka + 4 * g) * esz;
  int boff[PT];
#pragma unroll
  for (int pt = 0; pt < PT; ++pt) boff[pt] = ((pt * 16 + li) * I * Kb + 4 * g) * esz;
  bool ma[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) ma[u] = (KC - 1) * 16 + 4 * g + u < Ka;
  const bool afull = (Ka & 15) == 0;
  const TTC_LDS float* inl = In + li * ip + 4 * g;

  f32x4 bx0[KC], bx1[KC], gv[PT];
  raw_t br0[kDirect ? 1 : KC], br1[kDirect ? 1 : KC], gvn[PT];
  // G_A rows of mode index ii for both tiles (into the operands for FP32)
  auto load_a = [&](int ii) {
    const CoreRes ra = core_rsrc(op.ga, (long)ii * Ka, ta, esz);
#pragma unroll
    for (int kc = 0; kc < KC; ++kc) {
      if constexpr (kDirect) {
        bx0[kc] = R4::to_f32(R4::load(ra, aoff0 + kc * 16 * esz));
        bx1[kc] = R4::to_f32(R4::load(ra, aoff1 + kc * 16 * esz));
      } else {
        br0[kc] = R4::load(ra, aoff0 + kc * 16 * esz);
        br1[kc] = R4::load(ra, aoff1 + kc * 16 * esz);
      }
    }
  };
  // the loaded G_A rows as masked FP32 operands
  auto finish_a = [&]() {
#pragma unroll
    for (int kc = 0; kc < KC; ++kc) {
      const bool last = kc == KC - 1 && !afull;
      if constexpr (kDirect) {
        if (last) {
          bx0[kc] = R4::to_f32(bx0[kc], ma);
          bx1[kc] = R4::to_f32(bx1[kc], ma);
        }
      } else {
        bx0[kc] = last ? R4::to_f32(br0[kc], ma) : R4::to_f32(br0[kc]);
        bx1[kc] = last ? R4::to_f32(br1[kc], ma) : R4::to_f32(br1[kc]);
      }
    }
  };
  {
    load_a(0);
    const CoreRes rb = core_rsrc(op.gb, 0, tb, esz);
#pragma unroll
    for (int pt = 0; pt < PT; ++pt) gvn[pt] = R4::load(rb, boff[pt]);
    bool mb[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) mb[v] = 4 * g + v < Kb;
    finish_a();
#pragma unroll
    for (int pt = 0; pt < PT; ++pt) gv[pt] = R4::to_f32(gvn[pt], mb);
    __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
  }
  int i = 0, qt = 0;
  for (;;) {
    int ni = i, nq = qt + 1;
    if (nq == QT) {
      nq = 0;
      ni = i + 1;
    }
    const bool more = ni < I;
    if (more) {
      const CoreRes rb = core_rsrc(op.gb, (long)ni * Kb + nq * 16, tb, esz);
#pragma unroll
      for (int pt = 0; pt < PT; ++pt) gvn[pt] = R4::load(rb, boff[pt]);
    }
    f32x4 st0 = {0.f, 0.f, 0.f, 0.f}, st1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kc = 0; kc < KC; ++kc) {
      const f32x4 av = *reinterpret_cast<const TTC_LDS f32x4*>(inl + qt * 16 * ip + kc * 16);
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        st0 = mfma4(av[w], bx0[kc][w], st0);
        st1 = mfma4(av[w], bx1[kc][w], st1);
      }
    }
    // G_A rows of the next mode index (this slice's stage 1 was their last use)
    const bool reload = more && nq == 0;
    if (reload) load_a(ni);
#pragma unroll
    for (int pt = 0; pt < PT; ++pt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        acc0[pt] = mfma4(st0[v], gv[pt][v], acc0[pt]);
        acc1[pt] = mfma4(st1[v], gv[pt][v], acc1[pt]);
      }
    if (!more) break;
    if (nq * 16 + 16 <= Kb) {
#pragma unroll
      for (int pt = 0; pt < PT; ++pt) gv[pt] = R4::to_f32(gvn[pt]);
    } else {
      bool mb[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) mb[v] = nq * 16 + 4 * g + v < Kb;
#pragma unroll
      for (int pt = 0; pt < PT; ++pt) gv[pt] = R4::to_f32(gvn[pt], mb);
    }
    if (reload) finish_a();
    i = ni;
    qt = nq;
  }
}

// Both a-tiles at0, at1 of one wave over every mode index: in one pass for
// shapes that take one mode index per trip, else one pass per tile.
template <typename Tin, int KC, int PT>
__device__ __forceinline__ void lds_pair(const StepOp& op, const TTC_LDS float* In, int at0, int at1,
                                         f32x4 (&acc0)[SW_MAXT], f32x4 (&acc1)[SW_MAXT]) {
  if constexpr (TripWidth<KC, PT>::U == 1) {
    lds_tile2<Tin, KC, PT>(op, In, at0, at1, acc0, acc1);
  } else {
    lds_tile<Tin, KC, PT>(op, In, at0, 0, 1, acc0);
    lds_tile<Tin, KC, PT>(op, In, at1, 0, 1, acc1);
  }
}

template <typename Tin, int KC>
__device__ __forceinline__ void lds_pair_p(const StepOp& op, const TTC_LDS float* In, int at0, int at1,
                                           f32x4 (&acc0)[SW_MAXT], f32x4 (&acc1)[SW_MAXT]) {
  switch ((op.Nb + 15) >> 4) {
    case 1: lds_pair<Tin, KC, 1>(op, In, at0, at1, acc0, acc1); break;
    case 2: lds_pair<Tin, KC, 2>(op, In, at0, at1, acc0, acc1); break;
    case 3: lds_pair<Tin, KC, 3>(op, In, at0, at1, acc0, acc1); break;
    case 4: lds_pair<Tin, KC, 4>(op, In, at0, at1, acc0, acc1); break;
    case 5: lds_pair<Tin, KC, 5>(op, In, at0, at1, acc0, acc1); break;
    case 6: lds_pair<Tin, KC, 6>(op, In, at0, at1, acc0, acc1); break;
    case 7: lds_pair<Tin, KC, 7>(op, In, at0, at1, acc0, acc1); break;
    default: lds_pair<Tin, KC, 8>(op, In, at0, at1, acc0, acc1); break;
  }
}

template <typename Tin>
__device__ __forceinline__ void lds_pair_v(const StepOp& op, const TTC_LDS float* In, int at0, int at1,
                                           f32x4 (&acc0)[SW_MAXT], f32x4 (&acc1)[SW_MAXT]) {
  switch ((op.Ka + 15) >> 4) {
    case 1: lds_pair_p<Tin, 1>(op, In, at0, at1, acc0, acc1); break;
    case 2: lds_pair_p<Tin, 2>(op, In, at0, at1, acc0, acc1); break;
    case 3: lds_pair_p<Tin, 3>(op, In, at0, at1, acc0, acc1); break;
    case 4: lds_pair_p<Tin, 4>(op, In, at0, at1, acc0, acc1); break;
    case 5: lds_pair_p<Tin, 5>(op, In, at0, at1, acc0, acc1); break;
    case 6: lds_pair_p<Tin, 6>(op, In, at0, at1, acc0, acc1); break;
    case 7: lds_pair_p<Tin, 7>(op, In, at0, at1, acc0, acc1); break;
    default: lds_pair_p<Tin, 8>(op, In, at0, at1, acc0, acc1); break;
  }
}

template <typename Tin, int KC>
__device__ __forceinline__ void lds_tile_p(const StepOp& op, const TTC_LDS float* In, int at, int s0, int S,
                                           f32x4 (&acc)[SW_MAXT]) {
  switch ((op.Nb + 15) >> 4) {
    case 1: lds_tile<Tin, KC, 1>(op, In, at, s0, S, acc); break;
    case 2: lds_tile<Tin, KC, 2>(op, In, at, s0, S, acc); break;
    case 3: lds_tile<Tin, KC, 3>(op, In, at, s0, S, acc); break;
    case 4: lds_tile<Tin, KC, 4>(op, In, at, s0, S, acc); break;
    case 5: lds_tile<Tin, KC, 5>(op, In, at, s0, S, acc); break;
    case 6: lds_tile<Tin, KC, 6>(op, In, at, s0, S, acc); break;
    case 7: lds_tile<Tin, KC, 7>(op, In, at, s0, S, acc); break;
    default: lds_tile<Tin, KC, 8>(op, In, at, s0, S, acc); break;
  }
}

template <typename Tin>
__device__ __forceinline__ void lds_tile_v(const StepOp& op, const TTC_LDS float* In, int at, int s0, int S,
                                           f32x4 (&acc)[SW_MAXT]) {
  switch ((op.Ka + 15) >> 4) {
    case 1: lds_tile_p<Tin, 1>(op, In, at, s0, S, acc); break;
    case 2: lds_tile_p<Tin, 2>(op, In, at, s0, S, acc); break;
    case 3: lds_tile_p<Tin, 3>(op, In, at, s0, S, acc); break;
    case 4: lds_tile_p<Tin, 4>(op, In, at, s0, S, acc); break;
    case 5: lds_tile_p<Tin, 5>(op, In, at, s0, S, acc); break;
    case 6: lds_tile_p<Tin, 6>(op, In, at, s0, S, acc); break;
    case 7: lds_tile_p<Tin, 7>(op, In, at, s0, S, acc); break;
    default: lds_tile_p<Tin, 8>(op, In, at, s0, S, acc); break;
  }
}

// Store (FIRST) or add the a-tile `at` of Out: acc[pt][v] is
// Out[at*16 + 4g + v, pt*16 + li].  native: Out^T layout (rows b, pitch
// lds_pitch(Ma)), one 16-byte write per tile; else Out layout (rows a,
// pitch lds_pitch(Nb)).  Entries outside Ma x Nb are written as zeros.  When
// adding, every old value is read before any is written, so the reads
// overlap instead of each waiting for the previous write.
template <bool FIRST>
__device__ __forceinline__ void lds_put_t(TTC_LDS float* Out, bool native, int Ma, int Nb, int at,
                                          const f32x4 (&acc)[SW_MAXT]) {
  const int lane = threadIdx.x & 63, li = lane & 15, g = lane >> 4;
  const int PT = (Nb + 15) >> 4;
  const int a0 = at * 16 + 4 * g;
  const int pitch = native ? lds_pitch(Ma) : lds_pitch(Nb);
  f32x4 v[SW_MAXT];
#pragma unroll
  for (int pt = 0; pt < SW_MAXT; ++pt) {
    const int b = pt * 16 + li;
#pragma unroll
    for (int u = 0; u < 4; ++u) v[pt][u] = (a0 + u < Ma && b < Nb) ? acc[pt][u] : 0.f;
  }
  if (native) {
    if (!FIRST) {
      f32x4 old[SW_MAXT];
#pragma unroll
      for (int pt = 0; pt < SW_MAXT; ++pt)
        if (pt < PT) old[pt] = *reinterpret_cast<TTC_LDS f32x4*>(Out + (pt * 16 + li) * pitch + a0);
#pragma unroll
      for (int pt = 0; pt < SW_MAXT; ++pt)
        if (pt < PT) v[pt] = v[pt] + old[pt];
    }
#pragma unroll
    for (int pt = 0; pt < SW_MAXT; ++pt)
      if (pt < PT) *reinterpret_cast<TTC_LDS f32x4*>(Out + (pt * 16 + li) * pitch + a0) = v[pt];
  } else {
    if (!FIRST) {
      float old[SW_MAXT][4];
#pragma unroll
      for (int pt = 0; pt < SW_MAXT; ++pt)
        if (pt < PT)
#pragma unroll
          for (int u = 0; u < 4; ++u) old[pt][u] = Out[(a0 + u) * pitch + pt * 16 + li];
#pragma unroll
      for (int pt = 0; pt < SW_MAXT; ++pt)
        if (pt < PT)
#pragma unroll
          for (int u = 0; u < 4; ++u) v[pt][u] += old[pt][u];
    }
#pragma unroll
    for (int pt = 0; pt < SW_MAXT; ++pt)
      if (pt < PT)
#pragma unroll
        for (int u = 0; u < 4; ++u) Out[(a0 + u) * pitch + pt * 16 + li] = v[pt][u];
  }
}

__device__ __forceinline__ void lds_put(TTC_LDS float* Out, bool native, int Ma, int Nb, int at,
                                        const f32x4 (&acc)[SW_MAXT], bool first) {
  if (first) lds_put_t<true>(Out, native, Ma, Nb, at, acc);
  else lds_put_t<false>(Out, native, Ma, Nb, at, acc);
}

// One step by the NW waves of the workgroup.  Output tiles (16 rows of a)
// go to waves round-robin; when there are few tiles the mode indices are
// split S ways too and the partial tiles are added in a fixed order
// (deterministic).  Ends with a workgroup barrier.
template <typename Tin, int NW>
__device__ __forceinline__ void lds_step(const StepOp& op, const TTC_LDS float* In, TTC_LDS float* Out, bool native) {
  const int RT = (op.Ma + 15) >> 4;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  int S = 1, best = ((RT + NW - 1) / NW) * op.I;
  for (int c = 2; c <= NW && c <= op.I; c *= 2) {
    const int cost = ((RT * c + NW - 1) / NW) * ((op.I + c - 1) / c);
    if (cost < best) {
      best = cost;
      S = c;
    }
  }
  const int items = RT * S, passes = (items + NW - 1) / NW;
  for (int it = 0; it < passes; ++it) {
    const int item = w + it * NW;
    const bool active = item < items;
    const int at = item % RT, s = item / RT;
    f32x4 acc[SW_MAXT];
#pragma unroll
    for (int t = 0; t < SW_MAXT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    if (active) lds_tile_v<Tin>(op, In, at, s, S, acc);
    for (int ss = 0; ss < S; ++ss) {
      if (active && s == ss) lds_put(Out, native, op.Ma, op.Nb, at, acc, ss == 0);
      __syncthreads();
    }
  }
}

// The same step with one LDS buffer: In is overwritten by Out.  Each wave
// keeps at most two output tiles (two passes) in registers until every wave
// has finished reading In, then the tiles are stored in the fixed order of
// their mode-index parts.  Halving the LDS a pair needs lets two workgroups
// share a compute unit, so one's step boundaries (drain, barriers, first
// loads) overlap the other's MFMAs.  Ends with a workgroup barrier.
template <typename Tin, int NW>
__device__ __forceinline__ void lds_step_inplace(const StepOp& op, TTC_LDS float* Buf, bool native) {
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
  f32x4 acc[SW_MAXT], keep[SW_MAXT];
  if (S == 1 && w + NW < items) {
    // two a-tiles, every mode index: one pass where the shape allows
#pragma unroll
    for (int t = 0; t < SW_MAXT; ++t) keep[t] = acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    lds_pair_v<Tin>(op, Buf, w, w + NW, keep, acc);
  } else {
#pragma unroll 1
    for (int it = 0; it < 2; ++it) {
      const int item = w + it * NW;
#pragma unroll
      for (int t = 0; t < SW_MAXT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
      if (item < items) lds_tile_v<Tin>(op, Buf, item % RT, item / RT, S, acc);
      if (it == 0) {
#pragma unroll
        for (int t = 0; t < SW_MAXT; ++t) keep[t] = acc[t];
      }
    }
  }
  __syncthreads();  // In fully read
  const int item0 = w, item1 = w + NW;
  for (int ss = 0; ss < S; ++ss) {
    if (item0 < items && item0 / RT == ss) lds_put(Buf, native, op.Ma, op.Nb, item0 % RT, keep, ss == 0);
    if (item1 < items && item1 / RT == ss) lds_put(Buf, native, op.Ma, op.Nb, item1 % RT, acc, ss == 0);
    __syncthreads();
  }
}

// Per-thread part of <X, Y> = sum_i sum_p' T[i, p'] G_y^(0)[0, i, p'] with
// T = G_x^(0)[0, :, :] . V_1 (an I x P1 product, K = R1) and V_1 stored
// transposed in LDS (rows p', pitch lds_pitch(R1)); products and sums in FP64.
template <typename Tin, int KC, int NW>
__device__ __forceinline__ double lds_final_k(const void* gx0, const void* gy0, int I, int R1, int P1,
                                              const TTC_LDS float* V) {
  typedef Raw4<Tin> R4;
  constexpr int esz = sizeof(Tin);
  const int lane = threadIdx.x & 63, li = lane & 15, g = lane >> 4;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int MT = (I + 15) >> 4, NTl = (P1 + 15) >> 4, vp = lds_pitch(R1);
  const CoreRes rx = core_rsrc(gx0, 0, (long)I * R1, esz);
  const TTC_GLOBAL Tin* gy = gptr<Tin>(gy0);
  double s = 0.0;
  for (int item = w; item < MT * NTl; item += NW) {
    const int mt = item % MT, nt = item / MT;
    const int xoff = ((mt * 16 + li) * R1 + 4 * g) * esz;
    const TTC_LDS float* vl = V + (nt * 16 + li) * vp + 4 * g;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kc = 0; kc < KC; ++kc) {
      const typename R4::type a = R4::load(rx, xoff + kc * 16 * esz);
      const f32x4 b = *reinterpret_cast<const TTC_LDS f32x4*>(vl + kc * 16);
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

template <typename Tin, int NW>
__device__ __forceinline__ double lds_final(const void* gx0, const void* gy0, int I, int R1, int P1,
                                            const TTC_LDS float* V) {
  switch ((R1 + 15) >> 4) {
    case 1: return lds_final_k<Tin, 1, NW>(gx0, gy0, I, R1, P1, V);
    case 2: return lds_final_k<Tin, 2, NW>(gx0, gy0, I, R1, P1, V);
    case 3: return lds_final_k<Tin, 3, NW>(gx0, gy0, I, R1, P1, V);
    case 4: return lds_final_k<Tin, 4, NW>(gx0, gy0, I, R1, P1, V);
    case 5: return lds_final_k<Tin, 5, NW>(gx0, gy0, I, R1, P1, V);
    case 6: return lds_final_k<Tin, 6, NW>(gx0, gy0, I, R1, P1, V);
    case 7: return lds_final_k<Tin, 7, NW>(gx0, gy0, I, R1, P1, V);
    default: return lds_final_k<Tin, 8, NW>(gx0, gy0, I, R1, P1, V);
  }
}

}  // namespace ttc
