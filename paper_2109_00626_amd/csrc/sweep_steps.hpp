// One interface-sweep step as two chained MFMA products per mode index.
//
// Right to left (core k; V = V_{k+1} is Rn x Pn, result V_k is Rp x Pp):
//   S_i^T (Pn x Rp) = V^T . G_x^(k)[:, i, :]^T       (K = Rn)
//   V_k  (Rp x Pp) += S_i . G_y^(k)[:, i, :]^T        (K = Pn)
// Left to right (W = W_k is Rp x Pp, result W_{k+1} is Rn x Pn):
//   T_i  (Rp x Pn)  = W . G_y^(k)[:, i, :]             (K = Pp)
//   W_{k+1} (Rn x Pn) += G_x^(k)[:, i, :]^T . T_i      (K = Rp)
// The first product's accumulators are used directly as an operand of the
// second: an accumulator lane holds 4 rows of a 16x16 tile at one column,
// which is exactly a 16-wide K slice of the next MFMA if the K order is
// permuted to match (any order of a sum is valid).  So the per-mode
// intermediate never leaves registers and each core element is read once
// per workgroup, 4 contiguous elements per lane along the core's last
// (rank) index.
//
// Waves split the work by output tile (r-tiles right to left, p-tiles left
// to right) and, when there are more waves than tiles, by mode index; the
// partial sums of one tile are added in a fixed wave order through the
// output buffer (deterministic).  Interfaces are row-major with an odd row
// pitch (conflict-free column reads of LDS).
#pragma once
#include "ttc_device.hpp"
#include "ttc_internal.h"

namespace ttc {

__host__ __device__ __forceinline__ int iface_pitch(int P) { return (P & 1) ? P : P + 1; }

// Explicit address spaces: core pointers arrive through descriptors, so the
// compiler cannot prove they are global and would emit flat loads (which
// wait on both the vector-memory and LDS counters and serialise the loop).
// (The host compilation pass only parses these device functions.)
#if defined(__HIP_DEVICE_COMPILE__)
#define TTC_GLOBAL __attribute__((address_space(1)))
#define TTC_LDS __attribute__((address_space(3)))
#else
#define TTC_GLOBAL
#define TTC_LDS
#endif
template <typename T>
__device__ __forceinline__ const TTC_GLOBAL T* gptr(const void* p) {
  return (const TTC_GLOBAL T*)(p);
}
template <typename T>
__device__ __forceinline__ const TTC_LDS T* lptr(const void* p) {
  return (const TTC_LDS T*)(p);
}
__device__ __forceinline__ bool in_lds(const void* p) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_is_shared(p);
#else
  return false;
#endif
}

#define SW_MAXT 8  // up to 8 tiles of 16 per wave: ranks <= 128

// Four consecutive elements row[k..k+3] (zero beyond kmax or when !ok), as
// Tc.  Addresses are clamped into the row, so the loads are unconditional
// and the compiler can keep many of them in flight; `whole` (uniform) says
// the chunk is entirely inside the row, allowing one vector load.
template <typename Tin, typename Tc>
__device__ __forceinline__ void load4(const TTC_GLOBAL Tin* __restrict__ base, int off, int k, int kmax, bool ok,
                                      bool vec, Tc out[4], bool whole = false) {
  // element (off + k + u) of `base`, valid while k + u < kmax
  if (vec && whole) {
    if constexpr (sizeof(Tin) == 4) {
      const f32x4 v = *reinterpret_cast<const TTC_GLOBAL f32x4*>(base + (off + k));
#pragma unroll
      for (int u = 0; u < 4; ++u) out[u] = ok ? (Tc)v[u] : (Tc)0;
      return;
    } else if constexpr (sizeof(Tin) == 2) {
      const uint2 v = *reinterpret_cast<const TTC_GLOBAL uint2*>(base + (off + k));
      out[0] = ok ? (Tc)bf16_to_f32((uint16_t)(v.x & 0xFFFFu)) : (Tc)0;
      out[1] = ok ? (Tc)bf16_to_f32((uint16_t)(v.x >> 16)) : (Tc)0;
      out[2] = ok ? (Tc)bf16_to_f32((uint16_t)(v.y & 0xFFFFu)) : (Tc)0;
      out[3] = ok ? (Tc)bf16_to_f32((uint16_t)(v.y >> 16)) : (Tc)0;
      return;
    }
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int kk = min(k + u, kmax - 1);
    const Tc v = cvt<Tc>(base[off + kk]);
    out[u] = (ok && k + u < kmax) ? v : (Tc)0;
  }
}

// Elements base[off + k0 + K(g, v)] for v = 0..3, K the accumulator row map.
template <typename Tin, typename Tc>
__device__ __forceinline__ void load_acc_k(const TTC_GLOBAL Tin* __restrict__ base, int off, int k0, int g, int kmax,
                                           bool ok, bool vec, Tc out[4], bool whole = false) {
  if constexpr (sizeof(Tc) == 4) {
    load4<Tin, Tc>(base, off, k0 + 4 * g, kmax, ok, vec, out, whole);  // K(g, v) = 4g + v
  } else {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int k = k0 + Mfma<Tc>::row(g, v);
      const Tc x = cvt<Tc>(base[off + min(k, kmax - 1)]);
      out[v] = (ok && k < kmax) ? x : (Tc)0;
    }
  }
}

// Vectorised loads need 4-element rows at 4-element boundaries.
template <typename Tin>
__device__ __forceinline__ bool vec_ok(const void* base, int rowlen) {
  const uintptr_t a = reinterpret_cast<uintptr_t>(base);
  return (rowlen % 4 == 0) && (a % (4 * sizeof(Tin)) == 0);
}

// Accumulate the contribution of mode indices i = s, s + S, ... to the
// r-tile rt of V_k (right to left): one 16-column slice of S_i^T at a time
// (runtime loop over qt), each fed straight into every output p-tile.
// KC (the number of 16-wide chunks of R_{k+1}) is a template constant, so
// the chunk loops are unrolled without guards: the lane's whole G_x row of a
// mode index and a whole column of V are requested before their MFMAs, and
// the G_y operands of the second product before the first product.
template <typename Tin, typename Tc, int KC, typename VPtr>
__device__ __forceinline__ void rl_tile_k(const TTDev& x, const TTDev& y, int k, VPtr V, int ldv, int rt, int s,
                                          int S, typename Mfma<Tc>::acc (&acc)[SW_MAXT]) {
  typedef typename Mfma<Tc>::acc acc_t;
  const int Rp = x.ranks[k], Rn = x.ranks[k + 1];
  const int Pp = y.ranks[k], Pn = y.ranks[k + 1];
  const int I = x.modes[k];
  const TTC_GLOBAL Tin* Gx = gptr<Tin>(x.cores[k]);
  const TTC_GLOBAL Tin* Gy = gptr<Tin>(y.cores[k]);
  const bool vx = vec_ok<Tin>(x.cores[k], Rn), vy = vec_ok<Tin>(y.cores[k], Pn);
  const int lane = threadIdx.x & 63, li = lane & 15, g = lane >> 4;
  const int PT = (Pp + 15) >> 4, QT = (Pn + 15) >> 4;
  const int r = rt * 16 + li;
  const bool rok = r < Rp;
  const int gx_row0 = (rok ? r : 0) * I * Rn;  // element offset of G_x[r, 0, 0]
  for (int i = s; i < I; i += S) {
    Tc bx[KC][4];
#pragma unroll
    for (int kc = 0; kc < KC; ++kc)
      load4<Tin, Tc>(Gx, gx_row0 + i * Rn, kc * 16 + 4 * g, Rn, rok, vx, bx[kc], kc * 16 + 16 <= Rn);
#pragma unroll 1
    for (int qt = 0; qt < QT; ++qt) {
      Tc gb[SW_MAXT][4];
#pragma unroll
      for (int pt = 0; pt < SW_MAXT; ++pt) {
        if (pt < PT) {
          const int p = pt * 16 + li;
          const bool pok = p < Pp;
          load_acc_k<Tin, Tc>(Gy, ((pok ? p : 0) * I + i) * Pn, qt * 16, g, Pn, pok, vy, gb[pt],
                              qt * 16 + 16 <= Pn);
        }
      }
      // S_i^T[p' in tile qt, r] = sum_r'' V[r'', p'] G_x[r, i, r'']
      const int pc = qt * 16 + li;
      const bool pcok = pc < Pn;
      const int pcc = min(pc, Pn - 1);
      Tc av[KC][4];
#pragma unroll
      for (int kc = 0; kc < KC; ++kc)
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int kk = kc * 16 + 4 * g + u;
          const Tc xv = V[min(kk, Rn - 1) * ldv + pcc];
          av[kc][u] = (kk < Rn && pcok) ? xv : (Tc)0;
        }
      acc_t st = {0, 0, 0, 0};
#pragma unroll
      for (int kc = 0; kc < KC; ++kc)
#pragma unroll
        for (int u = 0; u < 4; ++u) st = Mfma<Tc>::step(av[kc][u], bx[kc][u], st);
      // V_k[r, p] += sum_p' S_i[r, p'] G_y[p, i, p']  (S_i^T accumulator as the A operand)
#pragma unroll
      for (int pt = 0; pt < SW_MAXT; ++pt) {
        if (pt < PT) {
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[pt] = Mfma<Tc>::step(st[v], gb[pt][v], acc[pt]);
        }
      }
    }
  }
}

template <typename Tin, typename Tc, typename VPtr>
__device__ __forceinline__ void rl_tile_v(const TTDev& x, const TTDev& y, int k, VPtr V, int ldv, int rt, int s,
                                          int S, typename Mfma<Tc>::acc (&acc)[SW_MAXT]) {
  switch ((x.ranks[k + 1] + 15) >> 4) {
    case 1: rl_tile_k<Tin, Tc, 1>(x, y, k, V, ldv, rt, s, S, acc); break;
    case 2: rl_tile_k<Tin, Tc, 2>(x, y, k, V, ldv, rt, s, S, acc); break;
    case 3: rl_tile_k<Tin, Tc, 3>(x, y, k, V, ldv, rt, s, S, acc); break;
    case 4: rl_tile_k<Tin, Tc, 4>(x, y, k, V, ldv, rt, s, S, acc); break;
    case 5: rl_tile_k<Tin, Tc, 5>(x, y, k, V, ldv, rt, s, S, acc); break;
    case 6: rl_tile_k<Tin, Tc, 6>(x, y, k, V, ldv, rt, s, S, acc); break;
    case 7: rl_tile_k<Tin, Tc, 7>(x, y, k, V, ldv, rt, s, S, acc); break;
    default: rl_tile_k<Tin, Tc, 8>(x, y, k, V, ldv, rt, s, S, acc); break;
  }
}

// V (the interface, R_{k+1} x P_{k+1}) may live in LDS or in global memory;
// the two cases are compiled separately so every load has a known space.
template <typename Tin, typename Tc>
__device__ __forceinline__ void rl_tile(const TTDev& x, const TTDev& y, int k, const Tc* V, int ldv, int rt, int s,
                                        int S, typename Mfma<Tc>::acc (&acc)[SW_MAXT]) {
  typedef typename Mfma<Tc>::acc acc_t;
#pragma unroll
  for (int t = 0; t < SW_MAXT; ++t) acc[t] = acc_t{0, 0, 0, 0};
  if (in_lds(V))
    rl_tile_v<Tin, Tc>(x, y, k, lptr<Tc>(V), ldv, rt, s, S, acc);
  else
    rl_tile_v<Tin, Tc>(x, y, k, gptr<Tc>(V), ldv, rt, s, S, acc);
}

// Accumulate mode indices i = s, s + S, ... into the p-tile pt of W_{k+1}
// (left to right): one 16-row slice of T_i at a time (runtime loop over
// rt), each fed straight into every output r-tile.  The lane's G_y column
// values of a mode index are loaded once, and the G_x operands of the second
// product are requested before the first product's MFMAs.
template <typename Tin, typename Tc, typename WPtr>
__device__ __forceinline__ void lr_tile_v(const TTDev& x, const TTDev& y, int k, WPtr W, int ldw, int pt, int s,
                                          int S, typename Mfma<Tc>::acc (&acc)[SW_MAXT]) {
  typedef typename Mfma<Tc>::acc acc_t;
  const int Rp = x.ranks[k], Rn = x.ranks[k + 1];
  const int Pp = y.ranks[k], Pn = y.ranks[k + 1];
  const int I = x.modes[k];
  const TTC_GLOBAL Tin* Gx = gptr<Tin>(x.cores[k]);
  const TTC_GLOBAL Tin* Gy = gptr<Tin>(y.cores[k]);
  const int lane = threadIdx.x & 63, li = lane & 15, g = lane >> 4;
  const int RT = (Rp + 15) >> 4, NT = (Rn + 15) >> 4, KP = (Pp + 15) >> 4;
  const int p = pt * 16 + li;
  const bool pok = p < Pn;
#pragma unroll
  for (int t = 0; t < SW_MAXT; ++t) acc[t] = acc_t{0, 0, 0, 0};
  for (int i = s; i < I; i += S) {
    Tc by[SW_MAXT][4];
#pragma unroll
    for (int kc = 0; kc < SW_MAXT; ++kc) {
      if (kc < KP) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int kk = kc * 16 + 4 * g + u;
          const Tc x = cvt<Tc>(Gy[(min(kk, Pp - 1) * I + i) * Pn + min(p, Pn - 1)]);
          by[kc][u] = (kk < Pp && pok) ? x : (Tc)0;
        }
      }
    }
#pragma unroll 1
    for (int rt = 0; rt < RT; ++rt) {
      Tc gv[4][SW_MAXT];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int kk = rt * 16 + Mfma<Tc>::row(g, v);
        const bool kok = kk < Rp;
        const int gx_off = ((kok ? kk : 0) * I + i) * Rn;
#pragma unroll
        for (int nt = 0; nt < SW_MAXT; ++nt) {
          if (nt < NT) {
            const int rr = nt * 16 + li;
            const Tc x = cvt<Tc>(Gx[gx_off + min(rr, Rn - 1)]);
            gv[v][nt] = (kok && rr < Rn) ? x : (Tc)0;
          }
        }
      }
      // T_i[r' in tile rt, p] = sum_p' W[r', p'] G_y[p', i, p]
      acc_t tacc = {0, 0, 0, 0};
      const int rr = rt * 16 + li;
      const bool rrok = rr < Rp;
      const int wrow = min(rr, Rp - 1) * ldw;
#pragma unroll
      for (int kc = 0; kc < SW_MAXT; ++kc) {
        if (kc < KP) {
          Tc aw[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int kk = kc * 16 + 4 * g + u;
            const Tc x = W[wrow + min(kk, Pp - 1)];
            aw[u] = (rrok && kk < Pp) ? x : (Tc)0;
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) tacc = Mfma<Tc>::step(aw[u], by[kc][u], tacc);
        }
      }
      // W_{k+1}[r, p] += sum_r' G_x[r', i, r] T_i[r', p]  (T_i accumulator as the B operand)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
#pragma unroll
        for (int nt = 0; nt < SW_MAXT; ++nt) {
          if (nt < NT) acc[nt] = Mfma<Tc>::step(gv[v][nt], tacc[v], acc[nt]);
        }
      }
    }
  }
}

template <typename Tin, typename Tc>
__device__ __forceinline__ void lr_tile(const TTDev& x, const TTDev& y, int k, const Tc* W, int ldw, int pt, int s,
                                        int S, typename Mfma<Tc>::acc (&acc)[SW_MAXT]) {
  if (in_lds(W))
    lr_tile_v<Tin, Tc>(x, y, k, lptr<Tc>(W), ldw, pt, s, S, acc);
  else
    lr_tile_v<Tin, Tc>(x, y, k, gptr<Tc>(W), ldw, pt, s, S, acc);
}

// Write (first) or add accumulator tiles.  fixed_is_row: tile `fixed` is a
// row tile and t runs over column tiles; otherwise the reverse.
template <typename Tc>
__device__ __forceinline__ void put_tiles(Tc* Out, int ldo, int M, int N, int fixed, bool fixed_is_row, int ntiles,
                                          const typename Mfma<Tc>::acc (&acc)[SW_MAXT], bool first) {
  const int lane = threadIdx.x & 63, li = lane & 15, g = lane >> 4;
#pragma unroll
  for (int t = 0; t < SW_MAXT; ++t) {
    if (t < ntiles) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int a = (fixed_is_row ? fixed : t) * 16 + Mfma<Tc>::row(g, v);
        const int b = (fixed_is_row ? t : fixed) * 16 + li;
        if (a < M && b < N) {
          Tc* q = Out + a * ldo + b;
          *q = first ? acc[t][v] : (Tc)(*q + acc[t][v]);
        }
      }
    }
  }
}

// Work split of one step: `tiles` output tiles over nw waves; with fewer
// tiles than waves the mode indices are split S ways as well.
struct StepSplit {
  int S, items, passes;
  __device__ StepSplit(int tiles, int nw) {
    S = tiles >= nw ? 1 : nw / tiles;
    items = tiles * S;
    passes = (items + nw - 1) / nw;
  }
};

// V_k from V_{k+1} (right to left).  V: Rn x Pn, pitch ldv.  Out: Rp x Pp, pitch ldo.
template <typename Tin, typename Tc>
__device__ __forceinline__ void rl_step_chain(const TTDev& x, const TTDev& y, int k, const Tc* V, int ldv, Tc* Out, int ldo) {
  typename Mfma<Tc>::acc acc[SW_MAXT];
  const int Rp = x.ranks[k], Pp = y.ranks[k];
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int RT = (Rp + 15) >> 4, PT = (Pp + 15) >> 4;
  const StepSplit sp(RT, nw);
  for (int it = 0; it < sp.passes; ++it) {
    const int item = w + it * nw;
    const bool active = item < sp.items;
    const int rt = item % RT, s = item / RT;
    if (active) rl_tile<Tin, Tc>(x, y, k, V, ldv, rt, s, sp.S, acc);
    for (int ss = 0; ss < sp.S; ++ss) {
      if (active && s == ss) put_tiles<Tc>(Out, ldo, Rp, Pp, rt, true, PT, acc, ss == 0);
      __syncthreads();
    }
  }
}

// W_{k+1} from W_k (left to right).  W: Rp x Pp, pitch ldw.  Out: Rn x Pn, pitch ldo.
template <typename Tin, typename Tc>
__device__ __forceinline__ void lr_step_chain(const TTDev& x, const TTDev& y, int k, const Tc* W, int ldw, Tc* Out, int ldo) {
  typename Mfma<Tc>::acc acc[SW_MAXT];
  const int Rn = x.ranks[k + 1], Pn = y.ranks[k + 1];
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int PT = (Pn + 15) >> 4, NT = (Rn + 15) >> 4;
  const StepSplit sp(PT, nw);
  for (int it = 0; it < sp.passes; ++it) {
    const int item = w + it * nw;
    const bool active = item < sp.items;
    const int pt = item % PT, s = item / PT;
    if (active) lr_tile<Tin, Tc>(x, y, k, W, ldw, pt, s, sp.S, acc);
    for (int ss = 0; ss < sp.S; ++ss) {
      if (active && s == ss) put_tiles<Tc>(Out, ldo, Rn, Pn, pt, false, NT, acc, ss == 0);
      __syncthreads();
    }
  }
}

}  // namespace ttc
