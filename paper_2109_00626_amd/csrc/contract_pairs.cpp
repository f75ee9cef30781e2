// Contraction of X's modes a1..a2 with Y's modes b1..b2 (consecutive blocks
// of equal length, pairwise equal sizes, anywhere in X and Y; eq. (8) once
// per pair, Def. 6): the two-sided transfer T of the blocks, and the
// junction, natural-order TT or dense output built from it.
//
// With a, b X's bonds before and after its block and g, d Y's, the result
// in eq. (8)'s mode order (X's free modes, then Y's) is
//   Z = sum XL[.., a] T[(a, g), (b, d)] XR[b, ..] YL[.., g] YR[d, ..].
// Natural-order TT: XL's cores are copied; the first XR core absorbs T and
// starts carrying q = (g, d) (Q = |g| |d|) through the rest of XR; YL's cores
// carry q on, and YL's last core contracts g with its right bond and passes
// d on to YR, whose cores are copied.  Without XR, XL's last core absorbs T;
// with X fully contracted, T is absorbed into YL's last core (or YR's first).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "ttc_layer.h"

namespace ttc {
ttc_status fail(ttc_status s, const std::string& msg);
hipError_t launch_transfer_first(ttc_dtype dt, const void* gx, const void* gy, int ka, int kg, int n, int kb,
                                 int kd, bool dab, void* E, hipStream_t s);
hipError_t launch_widen(const void* src, float* dst, long n, hipStream_t s);
hipError_t launch_transfer_step(ttc_dtype dt, const void* E, const void* gx, const void* gy, long rows, int ka1,
                                int kg1, int n, int kb, int kd, void* F, void* Eout, hipStream_t s);
}  // namespace ttc
using namespace ttc;

#define CP_TRY(expr)             \
  do {                           \
    ttc_status _s = (expr);      \
    if (_s != TTC_OK) return _s; \
  } while (0)
#define CP_HIP(expr)                                                                                     \
  do {                                                                                                   \
    hipError_t _e = (expr);                                                                              \
    if (_e != hipSuccess) return fail(TTC_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)

namespace {

// Largest transfer matrix or intermediate (elements) the path takes.
const long kMaxTransferElems = 1L << 28;

// A relayout-map radix larger than any row or column index: that digit is
// the whole index (and the next digit is zero).
const int kWhole = 1 << 30;

ttc_status check_one(const ttc_tt* t, const char* name) {
  if (!t) return fail(TTC_ERR_NULL, std::string(name) + " is NULL");
  if (t->order < 1 || t->order > TTC_MAX_ORDER) return fail(TTC_ERR_SHAPE, std::string(name) + ": order outside [1, 32]");
  if (!t->modes || !t->ranks || !t->cores) return fail(TTC_ERR_NULL, std::string(name) + ": NULL descriptor array");
  if (t->dtype != TTC_F64 && t->dtype != TTC_F32 && t->dtype != TTC_BF16)
    return fail(TTC_ERR_DTYPE, std::string(name) + ": unknown dtype");
  if (t->ranks[0] != 1 || t->ranks[t->order] != 1)
    return fail(TTC_ERR_RANK, std::string(name) + ": boundary ranks must be 1");
  for (int k = 0; k < t->order; ++k) {
    if (t->modes[k] < 1) return fail(TTC_ERR_SHAPE, std::string(name) + ": mode size < 1");
    if (t->ranks[k] < 1) return fail(TTC_ERR_RANK, std::string(name) + ": rank < 1");
    if (!t->cores[k]) return fail(TTC_ERR_NULL, std::string(name) + ": NULL core pointer");
    if ((double)t->ranks[k] * t->modes[k] * t->ranks[k + 1] >= 2147483647.0)
      return fail(TTC_ERR_SHAPE, std::string(name) + ": core too large");
  }
  return TTC_OK;
}

// One output core of the natural form: a lift op on one source core.
struct NatCore {
  int op, r0, n, r1, d0, d1, kg, kd;
  const void* src;
};

struct PairsPlan {
  int a1 = 0, a2 = 0, b1 = 0, b2 = 0, L = 0;
  int ka = 1, kb = 1, kg = 1, kd = 1;
  bool all = false;
  long rows = 1;          // ka * kg
  long e_max = 1, f_max = 1;
  // FP32 / BF16 cores: the steps after the first pair are MFMA products
  // (BF16 cores widened to FP32 first, exactly); FP64: per-entry FMA sums
  bool mfma = false;
  long gx_max = 0, gy_max = 0, slab = 0;
  int Q = 1;              // carried bond of the natural form
  std::vector<NatCore> nat;
  std::vector<int> nmodes, nranks;
  size_t cs = 4;
};

ttc_status plan_pairs(const ttc_tt* x, const ttc_tt* y, const int32_t* xm, const int32_t* ym, int32_t n,
                      PairsPlan* P) {
  CP_TRY(check_one(x, "x"));
  CP_TRY(check_one(y, "y"));
  if (x->dtype != y->dtype) return fail(TTC_ERR_DTYPE, "x and y have different dtypes");
  if (!xm || !ym) return fail(TTC_ERR_NULL, "mode lists are NULL");
  if (n < 1) return fail(TTC_ERR_MODE, "no contracted pairs");
  const int N = x->order, M = y->order;
  for (int l = 0; l < n; ++l) {
    if (xm[l] < 0 || xm[l] >= N) return fail(TTC_ERR_MODE, "x mode index out of range");
    if (ym[l] < 0 || ym[l] >= M) return fail(TTC_ERR_MODE, "y mode index out of range");
    if (l > 0 && (xm[l] == xm[l - 1] || ym[l] == ym[l - 1])) return fail(TTC_ERR_MODE, "repeated mode index");
  }
  for (int l = 1; l < n; ++l)
    if (xm[l] != xm[l - 1] + 1 || ym[l] != ym[l - 1] + 1)
      return fail(TTC_ERR_UNSUPPORTED, "GPU path needs consecutive increasing positions on both sides");
  for (int l = 0; l < n; ++l)
    if (x->modes[xm[l]] != y->modes[ym[l]])
      return fail(TTC_ERR_SHAPE, "contracted modes differ in size (pair " + std::to_string(l) + ")");
  P->L = n;
  P->a1 = xm[0];
  P->a2 = xm[n - 1];
  P->b1 = ym[0];
  P->b2 = ym[n - 1];
  P->ka = x->ranks[P->a1];
  P->kb = x->ranks[P->a2 + 1];
  P->kg = y->ranks[P->b1];
  P->kd = y->ranks[P->b2 + 1];
  P->cs = x->dtype == TTC_F64 ? 8 : 4;
  P->all = P->a1 == 0 && P->a2 == N - 1 && P->b1 == 0 && P->b2 == M - 1;
  P->rows = (long)P->ka * P->kg;
  // transfer sizes along the block
  P->e_max = 1;
  P->f_max = 1;
  for (int l = 0; l < n; ++l) {
    const long kb = x->ranks[P->a1 + l + 1], kd = y->ranks[P->b1 + l + 1];
    P->e_max = std::max(P->e_max, P->rows * kb * kd);
    if (l > 0) {
      const long kg1 = y->ranks[P->b1 + l];
      P->f_max = std::max(P->f_max, P->rows * kg1 * x->modes[P->a1 + l] * kb);
    }
  }
  if (P->e_max > kMaxTransferElems || P->f_max > kMaxTransferElems)
    return fail(TTC_ERR_UNSUPPORTED, "transfer matrix of the blocks exceeds 2^28 elements");
  // (the products are batched over the rows (a, g): at most 65535 of them)
  P->mfma = x->dtype != TTC_F64 && n > 1 && P->rows <= 65535;
  if (P->mfma) {
    for (int l = 1; l < n; ++l) {
      const int mx = P->a1 + l, my = P->b1 + l;
      P->gx_max = std::max(P->gx_max, (long)x->ranks[mx] * x->modes[mx] * x->ranks[mx + 1]);
      P->gy_max = std::max(P->gy_max, (long)y->ranks[my] * y->modes[my] * y->ranks[my + 1]);
    }
    // split-K partial outputs of the second product (at most four, 32 MB)
    P->slab = std::min(4 * P->e_max, 8L << 20);
  }
  // natural form
  P->nat.clear();
  P->nmodes.clear();
  const bool xfree = P->a1 > 0 || P->a2 < N - 1;
  const bool yl = P->b1 > 0;
  auto add = [&](int op, const ttc_tt* t, int m, int d0, int d1, int kg, int kd) {
    NatCore c;
    c.op = op;
    c.r0 = t->ranks[m];
    c.n = t->modes[m];
    c.r1 = t->ranks[m + 1];
    c.d0 = d0;
    c.d1 = d1;
    c.kg = kg;
    c.kd = kd;
    c.src = t->cores[m];
    P->nat.push_back(c);
    P->nmodes.push_back(c.n);
  };
  if (xfree) {
    const int Q = P->kg * P->kd;
    P->Q = Q;
    const bool xr = P->a2 < N - 1;
    for (int m = 0; m < P->a1; ++m) {
      if (!xr && m == P->a1 - 1)
        add(LIFT_ABSORB_R, x, m, x->ranks[m], Q, 0, 0);
      else
        add(LIFT_COPY, x, m, x->ranks[m], x->ranks[m + 1], 0, 0);
    }
    for (int m = P->a2 + 1; m < N; ++m) {
      if (m == P->a2 + 1)
        add(LIFT_ABSORB_M, x, m, P->ka, x->ranks[m + 1] * Q, P->kg, P->kd);
      else
        add(LIFT_DELTA, x, m, x->ranks[m] * Q, x->ranks[m + 1] * Q, 0, 0);
    }
    for (int m = 0; m < P->b1; ++m) {
      if (m == P->b1 - 1)
        add(LIFT_DELTA_SPLIT, y, m, y->ranks[m] * Q, P->kd, P->kg, P->kd);
      else
        add(LIFT_DELTA, y, m, y->ranks[m] * Q, y->ranks[m + 1] * Q, 0, 0);
    }
    for (int m = P->b2 + 1; m < M; ++m) add(LIFT_COPY, y, m, y->ranks[m], y->ranks[m + 1], 0, 0);
  } else if (!P->all) {
    // X fully contracted: T (kg x kd) joins Y's two parts
    P->Q = yl ? P->kd : 1;
    for (int m = 0; m < P->b1; ++m) {
      if (m == P->b1 - 1)
        add(LIFT_ABSORB_R, y, m, y->ranks[m], P->kd, 0, 0);
      else
        add(LIFT_COPY, y, m, y->ranks[m], y->ranks[m + 1], 0, 0);
    }
    for (int m = P->b2 + 1; m < M; ++m) {
      if (!yl && m == P->b2 + 1)
        add(LIFT_ABSORB_L, y, m, 1, y->ranks[m + 1], 0, 0);
      else
        add(LIFT_COPY, y, m, y->ranks[m], y->ranks[m + 1], 0, 0);
    }
  }
  P->nranks.clear();
  if (!P->nat.empty()) {
    P->nranks.push_back(P->nat[0].d0);
    for (const auto& c : P->nat) P->nranks.push_back(c.d1);
  }
  return TTC_OK;
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

struct PairsWs {
  size_t e0 = 0, e1 = 0, f = 0, cores = 0, inner = 0, total = 0;
  size_t slab = 0, gx = 0, gy = 0;  // MFMA steps: split-K slabs; BF16 cores widened to FP32
  std::vector<size_t> core_off;
};

ttc_status size_ws(const ttc_tt* x, const ttc_tt* y, const PairsPlan& P, ttc_form form, PairsWs* W) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  if (P.all) {
    size_t need = 0;
    CP_TRY(tt_contract_inner_query(x, y, TTC_PREC_AUTO, &need));
    W->inner = take(need);
  } else {
    W->e0 = take(P.e_max * P.cs);
    W->e1 = take(P.e_max * P.cs);
    W->f = take(P.f_max * P.cs);
    if (P.mfma) {
      W->slab = take(P.slab * 4);
      if (x->dtype == TTC_BF16) {
        W->gx = take(P.gx_max * 4);
        W->gy = take(P.gy_max * 4);
      }
    }
    if (form == TTC_DENSE) {
      W->core_off.clear();
      for (const auto& c : P.nat) W->core_off.push_back(take((size_t)c.d0 * c.n * c.d1 * P.cs));
    }
  }
  W->total = off;
  return TTC_OK;
}

}  // namespace

extern "C" {

ttc_status tt_contract_pairs_query(const ttc_tt* x, const ttc_tt* y, const int32_t* xmodes, const int32_t* ymodes,
                                   int32_t n_pairs, ttc_form form, int32_t* out_order, int32_t* out_modes,
                                   int32_t* out_ranks, int64_t* out_elems, size_t* ws_bytes) {
  PairsPlan P;
  CP_TRY(plan_pairs(x, y, xmodes, ymodes, n_pairs, &P));
  if (form != TTC_JUNCTION && form != TTC_NATURAL_TT && form != TTC_DENSE)
    return fail(TTC_ERR_UNSUPPORTED, "unknown form");
  int order = 0;
  int64_t elems = 1;
  if (P.all) {
    order = 0;
  } else if (form == TTC_JUNCTION) {
    order = 2;
    elems = P.rows * (int64_t)P.kb * P.kd;
    if (out_ranks) {
      out_ranks[0] = (int32_t)P.rows;
      out_ranks[1] = P.kb * P.kd;
    }
  } else {
    order = (int)P.nat.size();
    if (form == TTC_NATURAL_TT) {
      elems = 0;
      for (const auto& c : P.nat) elems += (int64_t)c.d0 * c.n * c.d1;
    } else {
      for (const auto& c : P.nat) {
        if (c.d0 > 64 || c.d1 > 64) return fail(TTC_ERR_UNSUPPORTED, "dense form limited to natural ranks <= 64");
        elems *= c.n;
      }
      if (elems > (1L << 31)) return fail(TTC_ERR_UNSUPPORTED, "dense form limited to 2^31 entries");
    }
    if (out_modes)
      for (int m = 0; m < order; ++m) out_modes[m] = P.nmodes[m];
    if (out_ranks)
      for (int m = 0; m <= order; ++m) out_ranks[m] = P.nranks[m];
  }
  PairsWs W;
  CP_TRY(size_ws(x, y, P, form, &W));
  if (out_order) *out_order = order;
  if (out_elems) *out_elems = elems;
  if (ws_bytes) *ws_bytes = W.total;
  return TTC_OK;
}

ttc_status tt_contract_pairs(const ttc_tt* x, const ttc_tt* y, const int32_t* xmodes, const int32_t* ymodes,
                             int32_t n_pairs, ttc_form form, void* out_junction, const ttc_tt* out_tt,
                             void* out_dense, double* out_scalar, void* d_ws, size_t ws_bytes, void* stream) {
  size_t need = 0;
  int32_t order = 0;
  int64_t elems = 0;
  CP_TRY(tt_contract_pairs_query(x, y, xmodes, ymodes, n_pairs, form, &order, nullptr, nullptr, &elems, &need));
  if (need > ws_bytes) return fail(TTC_ERR_WORKSPACE, "workspace smaller than tt_contract_pairs_query size");
  if (need && !d_ws) return fail(TTC_ERR_NULL, "d_ws is NULL");
  PairsPlan P;
  CP_TRY(plan_pairs(x, y, xmodes, ymodes, n_pairs, &P));
  PairsWs W;
  CP_TRY(size_ws(x, y, P, form, &W));
  hipStream_t s = (hipStream_t)stream;
  char* ws = static_cast<char*>(d_ws);
  if (P.all) {
    if (!out_scalar) return fail(TTC_ERR_NULL, "out_scalar is NULL (every position contracted)");
    size_t inner_need = 0;
    CP_TRY(tt_contract_inner_query(x, y, TTC_PREC_AUTO, &inner_need));
    return tt_contract_inner(x, y, TTC_PREC_AUTO, out_scalar, inner_need ? ws + W.inner : nullptr, inner_need,
                             stream);
  }
  if (form == TTC_JUNCTION && !out_junction) return fail(TTC_ERR_NULL, "out_junction is NULL");
  if (form == TTC_DENSE && !out_dense) return fail(TTC_ERR_NULL, "out_dense is NULL");
  std::vector<void*> dst(P.nat.size(), nullptr);
  if (form == TTC_NATURAL_TT) {
    if (!out_tt || !out_tt->cores) return fail(TTC_ERR_NULL, "out_tt is NULL");
    if (out_tt->order != (int)P.nat.size()) return fail(TTC_ERR_SHAPE, "out_tt order differs from the query's");
    for (size_t m = 0; m < P.nat.size(); ++m) {
      if (out_tt->modes[m] != P.nmodes[m] || out_tt->ranks[m] != P.nranks[m] ||
          out_tt->ranks[m + 1] != P.nranks[m + 1])
        return fail(TTC_ERR_SHAPE, "out_tt shape differs from the query's");
      if (!out_tt->cores[m]) return fail(TTC_ERR_NULL, "NULL output core");
      dst[m] = out_tt->cores[m];
    }
  } else if (form == TTC_DENSE) {
    for (size_t m = 0; m < P.nat.size(); ++m) dst[m] = ws + W.core_off[m];
  }
  // transfer sweep over the blocks
  const ttc_dtype dt = x->dtype;
  void* E = ws + W.e0;
  void* E2 = ws + W.e1;
  void* F = ws + W.f;
  CP_HIP(launch_transfer_first(dt, x->cores[P.a1], y->cores[P.b1], P.ka, P.kg, x->modes[P.a1], x->ranks[P.a1 + 1],
                               y->ranks[P.b1 + 1], P.mfma, E, s));
  for (int l = 1; l < P.L; ++l) {
    const int mx = P.a1 + l, my = P.b1 + l;
    const int ka1 = x->ranks[mx], kg1 = y->ranks[my], nm = x->modes[mx], kb = x->ranks[mx + 1],
              kd = y->ranks[my + 1];
    if (!P.mfma) {
      CP_HIP(launch_transfer_step(dt, E, x->cores[mx], y->cores[my], P.rows, ka1, kg1, nm, kb, kd, F, E2, s));
      std::swap(E, E2);
      continue;
    }
    // E holds [g'][(a, g)][a'] (kg1 x rows x ka1)
    const float* gx = reinterpret_cast<const float*>(x->cores[mx]);
    const float* gy = reinterpret_cast<const float*>(y->cores[my]);
    if (dt == TTC_BF16) {
      float* wx = reinterpret_cast<float*>(ws + W.gx);
      float* wy = reinterpret_cast<float*>(ws + W.gy);
      CP_HIP(launch_widen(x->cores[mx], wx, (long)ka1 * nm * kb, s));
      CP_HIP(launch_widen(y->cores[my], wy, (long)kg1 * nm * kd, s));
      gx = wx;
      gy = wy;
    }
    const long rb = P.rows * kb;
    // per row (a, g), batched over the rows:
    //   F[(g', i)][(a, g)][b] = sum_a' E[g'][(a, g)][a'] Gx[a'][(i, b)]
    // (the store places the row's g' x (i, b) block at its slots of F)
    IdxMap fmap;
    fmap.mr0 = kWhole;
    fmap.mr1 = kWhole;
    fmap.ms0 = (long)nm * rb;
    fmap.ms1 = 0;
    fmap.ms2 = 0;
    fmap.nr0 = kb;
    fmap.ns0 = 1;
    fmap.ns1 = rb;
    CP_TRY(gemm_f32_batched(true, reinterpret_cast<const float*>(E), P.rows * ka1, ka1, false, gx, (long)nm * kb, 0,
                            reinterpret_cast<float*>(F), 0, kb, kg1, nm * kb, ka1, (int)P.rows, s, &fmap));
    // then one product over all rows:
    //   E'[d][((a, g), b)] = sum_{(g', i)} Gy[(g', i)][d] F[(g', i)][((a, g), b)]
    // in the next pair's layout [d][(a, g)][b], or after the last pair as
    // T[(a, g)][(b, d)]
    float* Eo = reinterpret_cast<float*>(E2);
    if (l < P.L - 1) {
      CP_TRY(gemm_f32(false, gy, kd, false, reinterpret_cast<const float*>(F), rb, Eo, rb, kd, (int)rb, kg1 * nm,
                      reinterpret_cast<float*>(ws + W.slab), (size_t)P.slab, s, nullptr));
    } else {
      IdxMap tmap;
      tmap.mr0 = kWhole;
      tmap.mr1 = kWhole;
      tmap.ms0 = 1;
      tmap.ms1 = 0;
      tmap.ms2 = 0;
      tmap.nr0 = kb;
      tmap.ns0 = kd;
      tmap.ns1 = (long)kb * kd;
      CP_TRY(gemm_f32(false, gy, kd, false, reinterpret_cast<const float*>(F), rb, Eo, 0, kd, (int)rb, kg1 * nm,
                      nullptr, 0, s, &tmap));
    }
    std::swap(E, E2);
  }
  if (form == TTC_JUNCTION) {
    CP_HIP(hipMemcpyAsync(out_junction, E, (size_t)elems * P.cs, hipMemcpyDeviceToDevice, s));
    return TTC_OK;
  }
  LiftArgs la;
  std::memset(&la, 0, sizeof(la));
  la.Q = P.Q;
  la.kr = 0;
  la.K = E;
  int lines = 0;
  for (size_t m = 0; m < P.nat.size(); ++m) {
    const NatCore& c = P.nat[m];
    LiftCore& o = la.c[m];
    o.op = c.op;
    o.r0 = c.r0;
    o.n = c.n;
    o.r1 = c.r1;
    o.d0 = c.d0;
    o.d1 = c.d1;
    o.kg = c.kg;
    o.kd = c.kd;
    o.src = c.src;
    o.dst = dst[m];
    lines += c.d0 * c.n;
  }
  la.ncores = (int)P.nat.size();
  CP_HIP(launch_lift(dt, la, lines, s));
  if (form == TTC_DENSE) {
    DenseArgs da;
    std::memset(&da, 0, sizeof(da));
    da.t.order = (int)P.nat.size();
    for (size_t m = 0; m < P.nat.size(); ++m) {
      da.t.modes[m] = P.nmodes[m];
      da.t.cores[m] = dst[m];
    }
    for (size_t m = 0; m < P.nranks.size(); ++m) da.t.ranks[m] = P.nranks[m];
    da.numel = elems;
    da.out = out_dense;
    CP_HIP(launch_dense(dt == TTC_F64, da, s));
  }
  return TTC_OK;
}

}  // extern "C"
