// Host runtime behind the C ABI: argument validation (before any launch),
// shape bookkeeping, workspace sizing and kernel dispatch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "ttc_internal.h"

using namespace ttc;

namespace ttc {
thread_local std::string g_err;

ttc_status fail(ttc_status s, const std::string& msg) {
  g_err = msg;
  return s;
}
}  // namespace ttc

#define TTC_TRY(expr)                      \
  do {                                     \
    ttc_status _s = (expr);                \
    if (_s != TTC_OK) return _s;           \
  } while (0)

#define TTC_HIP(expr)                                                                             \
  do {                                                                                            \
    hipError_t _e = (expr);                                                                       \
    if (_e != hipSuccess) return fail(TTC_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)

namespace {

size_t elem_size(ttc_dtype d) { return d == TTC_F64 ? 8 : (d == TTC_F32 ? 4 : 2); }
// Interface / output element size: FP64 for FP64 inputs, FP32 otherwise.
size_t comp_size(ttc_dtype d) { return d == TTC_F64 ? 8 : 4; }
bool dtype_ok(int d) { return d == TTC_F64 || d == TTC_F32 || d == TTC_BF16; }

ttc_status ensure_init() {
  static std::atomic<bool> done[kMaxDevices];
  const hipError_t st = once_per_device(done, [] { return sweep_set_lds_limits(); });
  if (st != hipSuccess) return fail(TTC_ERR_HIP, std::string("kernel attribute setup: ") + hipGetErrorString(st));
  return TTC_OK;
}

ttc_status check_tt(const ttc_tt* t, const char* name, int max_order = TTC_MAX_ORDER) {
  if (!t) return fail(TTC_ERR_NULL, std::string(name) + " is NULL");
  if (t->order < 1 || t->order > max_order)
    return fail(TTC_ERR_SHAPE, std::string(name) + ": order " + std::to_string(t->order) + " outside [1, " +
                                   std::to_string(max_order) + "]");
  if (!t->modes || !t->ranks || !t->cores) return fail(TTC_ERR_NULL, std::string(name) + ": NULL descriptor array");
  if (!dtype_ok(t->dtype)) return fail(TTC_ERR_DTYPE, std::string(name) + ": unknown dtype");
  const int N = t->order;
  if (t->ranks[0] != 1 || t->ranks[N] != 1)
    return fail(TTC_ERR_RANK, std::string(name) + ": boundary ranks must be 1");
  for (int k = 0; k < N; ++k) {
    if (t->modes[k] < 1) return fail(TTC_ERR_SHAPE, std::string(name) + ": mode size < 1");
    if (t->ranks[k] < 1) return fail(TTC_ERR_RANK, std::string(name) + ": rank < 1");
    if (!t->cores[k]) return fail(TTC_ERR_NULL, std::string(name) + ": NULL core pointer");
    const double ne = (double)t->ranks[k] * t->modes[k] * t->ranks[k + 1];
    if (ne >= 2147483647.0) return fail(TTC_ERR_SHAPE, std::string(name) + ": core too large");
  }
  return TTC_OK;
}

ttc_status check_pair(const ttc_tt* x, const ttc_tt* y, int max_order = TTC_MAX_ORDER) {
  TTC_TRY(check_tt(x, "x", max_order));
  TTC_TRY(check_tt(y, "y", max_order));
  if (x->order != y->order) return fail(TTC_ERR_SHAPE, "x and y have different orders");
  if (x->dtype != y->dtype) return fail(TTC_ERR_DTYPE, "x and y have different dtypes");
  for (int k = 0; k < x->order; ++k)
    if (x->modes[k] != y->modes[k]) return fail(TTC_ERR_SHAPE, "x and y differ in mode " + std::to_string(k));
  return TTC_OK;
}

ttc_status check_prec(ttc_prec p, ttc_dtype d) {
  if (p == TTC_PREC_AUTO) return TTC_OK;
  if (d == TTC_F64 && p == TTC_PREC_F64) return TTC_OK;
  if (d != TTC_F64 && p == TTC_PREC_F32) return TTC_OK;
  return fail(TTC_ERR_UNSUPPORTED, "precision not available for this dtype");
}

TTDev to_dev(const ttc_tt* t) {
  TTDev d;
  std::memset(&d, 0, sizeof(d));
  d.order = t->order;
  for (int k = 0; k < t->order; ++k) {
    d.modes[k] = t->modes[k];
    d.cores[k] = t->cores[k];
  }
  for (int k = 0; k <= t->order; ++k) d.ranks[k] = t->ranks[k];
  return d;
}

// Bump allocator over the caller's workspace (sizing when base is null).
struct Arena {
  char* base;
  size_t off = 0;
  explicit Arena(void* b) : base((char*)b) {}
  void* take(size_t bytes) {
    off = (off + 255) & ~(size_t)255;
    void* p = base ? base + off : nullptr;
    off += bytes;
    return p;
  }
};

// LDS / intermediate sizing of a sweep over cores [k0, k1).
struct SweepSizing {
  int max_rp = 1;
  int tcap = 1;
  bool t_global = false;
  bool i_global = false;
  bool chain = false;
  size_t lds = 0;
  size_t t_block_bytes = 0;
  size_t i_block_bytes = 0;
};

// Interfaces and the per-mode intermediate go to LDS when they fit; what
// does not fit goes to a per-block slice of the workspace.  With every rank
// <= 128 the chained-MFMA steps are used: no intermediate buffer, and
// interfaces stored with an odd row pitch.
int iface_pitch_h(int P) { return (P & 1) ? P : P + 1; }

ttc_status size_sweep(const ttc_tt* x, const ttc_tt* y, int k0, int k1, SweepSizing* out, bool allow_chain = true) {
  const size_t cs = comp_size(x->dtype);
  long max_rp = 1, max_t = 1, max_I = 1;
  int max_rank = 1;
  for (int b = 0; b <= x->order; ++b) max_rank = std::max(max_rank, std::max(x->ranks[b], y->ranks[b]));
  const bool chain = allow_chain && max_rank <= 128;
  for (int b = k0; b <= k1; ++b)
    max_rp = std::max<long>(max_rp, (long)x->ranks[b] * (chain ? iface_pitch_h(y->ranks[b]) : y->ranks[b]));
  for (int k = k0; k < k1; ++k) {
    max_t = std::max<long>(max_t, (long)x->ranks[k] * y->ranks[k + 1]);
    max_I = std::max<long>(max_I, x->modes[k]);
  }
  const long budget = lds_limit_bytes() / (long)cs;
  SweepSizing s;
  s.max_rp = (int)max_rp;
  s.chain = chain;
  long lds_elems = 0;
  if (2 * max_rp <= budget) {
    lds_elems = 2 * max_rp;
  } else {
    s.i_global = true;
    s.i_block_bytes = (size_t)(2 * max_rp) * cs;
  }
  if (!chain) {
    const long left = budget - lds_elems;
    if (left >= max_t) {
      s.tcap = (int)std::min(left, max_t * max_I);
      lds_elems += s.tcap;
    } else {
      s.tcap = (int)(max_t * std::min<long>(max_I, 8));
      s.t_global = true;
      s.t_block_bytes = (size_t)s.tcap * cs;
    }
  }
  s.lds = (size_t)lds_elems * cs;
  *out = s;
  return TTC_OK;
}

enum BlockKind { BK_ALL, BK_PREFIX, BK_SUFFIX, BK_OTHER };

ttc_status classify(int N, const int32_t* modes, int n, BlockKind* kind, int* k) {
  if (n < 1) return fail(TTC_ERR_MODE, "empty mode list");
  if (!modes) return fail(TTC_ERR_NULL, "modes is NULL");
  std::vector<int> s(modes, modes + n);
  std::sort(s.begin(), s.end());
  for (int i = 0; i < n; ++i) {
    if (s[i] < 0 || s[i] >= N) return fail(TTC_ERR_MODE, "mode index out of range");
    if (i && s[i] == s[i - 1]) return fail(TTC_ERR_MODE, "repeated mode index");
  }
  bool prefix = true, suffix = true;
  for (int i = 0; i < n; ++i) {
    if (s[i] != i) prefix = false;
    if (s[i] != N - n + i) suffix = false;
  }
  if (n == N) {
    *kind = BK_ALL;
    *k = N;
  } else if (prefix) {
    *kind = BK_PREFIX;
    *k = n;
  } else if (suffix) {
    *kind = BK_SUFFIX;
    *k = N - n;
  } else {
    *kind = BK_OTHER;
    *k = -1;
  }
  return TTC_OK;
}

// Shape of the natural-order TT of a prefix / suffix contraction.
void natural_shape(const ttc_tt* x, const ttc_tt* y, BlockKind kind, int k, std::vector<int>* modes,
                   std::vector<int>* ranks) {
  const int N = x->order;
  modes->clear();
  ranks->clear();
  const int Q = y->ranks[k];
  if (kind == BK_PREFIX) {
    ranks->push_back(1);
    for (int m = k; m < N; ++m) {
      modes->push_back(x->modes[m]);
      ranks->push_back(x->ranks[m + 1] * Q);
    }
    for (int m = k; m < N; ++m) {
      modes->push_back(y->modes[m]);
      ranks->push_back(y->ranks[m + 1]);
    }
  } else {
    for (int m = 0; m < k; ++m) {
      modes->push_back(x->modes[m]);
      ranks->push_back(x->ranks[m]);
    }
    ranks->push_back(Q);
    for (int m = 0; m < k; ++m) modes->push_back(y->modes[m]);
    for (int m = 1; m < k; ++m) ranks->push_back(y->ranks[m] * Q);
    ranks->push_back(1);
  }
}

// Reversed, rank-transposed copies of cores [0, n) of X and Y in the
// workspace (core j of the copy is core n-1-j with its rank axes exchanged)
// and their descriptors: the right-to-left sweep of the copy is the
// left-to-right sweep of the original.  With a null arena base only sizes.
void reversed_pair(const ttc_tt* x, const ttc_tt* y, int n, Arena& ws, TTDev* xr, TTDev* yr, CoreRevArgs* ra) {
  const size_t esz = x->dtype == TTC_BF16 ? 2 : 4;
  std::memset(xr, 0, sizeof(*xr));
  std::memset(yr, 0, sizeof(*yr));
  std::memset(ra, 0, sizeof(*ra));
  xr->order = yr->order = n;
  ra->esz = (int)esz;
  const ttc_tt* t[2] = {x, y};
  TTDev* d[2] = {xr, yr};
  for (int q = 0; q < 2; ++q) {
    for (int j = 0; j < n; ++j) {
      const int m = n - 1 - j;
      const int R = t[q]->ranks[m], I = t[q]->modes[m], R1 = t[q]->ranks[m + 1];
      void* dst = ws.take((size_t)R * I * R1 * esz);
      d[q]->modes[j] = I;
      d[q]->cores[j] = dst;
      CoreRevItem& c = ra->c[ra->n++];
      c.src = t[q]->cores[m];
      c.dst = dst;
      c.R = R;
      c.I = I;
      c.R1 = R1;
    }
    for (int j = 0; j <= n; ++j) d[q]->ranks[j] = t[q]->ranks[n - j];
  }
}

bool lds_path(const ttc_tt* x, const ttc_tt* y) {
  return x->dtype != TTC_F64 && pair_lds_ok(to_dev(x), to_dev(y));
}

// Runs the junction sweep (prefix: W_k left to right; suffix: V_k right to left)
// into `kout` (compute type).
ttc_status run_junction(const ttc_tt* x, const ttc_tt* y, BlockKind kind, int k, void* kout, Arena& ws,
                        size_t ws_bytes, bool sizing, hipStream_t s, bool m16 = false) {
  if (lds_path(x, y)) {
    // one workgroup, interface in LDS; a prefix runs on the reversed block
    PairLdsArgs pa;
    std::memset(&pa, 0, sizeof(pa));
    CoreRevArgs ra;
    if (kind == BK_PREFIX) {
      reversed_pair(x, y, k, ws, &pa.side[0].x, &pa.side[0].y, &ra);
      pa.side[0].stop = 0;
    } else {
      pa.side[0].x = to_dev(x);
      pa.side[0].y = to_dev(y);
      pa.side[0].stop = k;
    }
    if (sizing) return TTC_OK;
    if (ws.off > ws_bytes) return fail(TTC_ERR_WORKSPACE, "workspace too small");
    pa.side[0].out = reinterpret_cast<float*>(kout);
    pa.m16 = m16;
    if (kind == BK_PREFIX) TTC_HIP(launch_core_reverse(ra, s));
    TTC_HIP(launch_pair_lds(x->dtype, pa, 1, s));
    return TTC_OK;
  }
  SweepSizing sz;
  const int k0 = kind == BK_PREFIX ? 0 : k, k1 = kind == BK_PREFIX ? k : x->order;
  TTC_TRY(size_sweep(x, y, k0, k1, &sz));
  void* tg = sz.t_global ? ws.take(sz.t_block_bytes) : nullptr;
  void* ig = sz.i_global ? ws.take(sz.i_block_bytes) : nullptr;
  if (sizing) return TTC_OK;
  if (ws.off > ws_bytes) return fail(TTC_ERR_WORKSPACE, "workspace too small");
  SweepArgs a;
  std::memset(&a, 0, sizeof(a));
  a.x = to_dev(x);
  a.y = to_dev(y);
  a.dir[0] = kind == BK_PREFIX ? 0 : 1;
  a.dir[1] = -1;
  a.stop[0] = k;
  a.out[0] = kout;
  a.max_rp = sz.max_rp;
  a.tcap = sz.tcap;
  a.t_global = tg;
  a.t_stride = sz.tcap;
  a.i_global = ig;
  a.i_stride = 2L * sz.max_rp;
  a.chain = sz.chain;
  TTC_HIP(launch_sweep(x->dtype, a, 1, sz.lds, s));
  return TTC_OK;
}

// Bidirectional inner product meeting at bond N/2.
// m16: BF16 cores on the BF16-MFMA steps (LDS path only).
ttc_status run_inner(const ttc_tt* x, const ttc_tt* y, double* d_out, Arena& ws, size_t ws_bytes, bool sizing,
                     hipStream_t s, bool m16 = false) {
  if (lds_path(x, y) && x->order >= 4) {
    // two half sweeps at once, one workgroup each, meeting at bond c: V_c right
    // to left over cores c..N-1, W_c as the right-to-left sweep of the
    // reversed, rank-transposed prefix (cores 0..c-1); then <X, Y> = sum W_c .* V_c
    const int c = x->order / 2;
    const size_t rp = (size_t)x->ranks[c] * y->ranks[c];
    void* W = ws.take(rp * sizeof(float));
    void* V = ws.take(rp * sizeof(float));
    PairLdsArgs pa;
    std::memset(&pa, 0, sizeof(pa));
    CoreRevArgs ra;
    reversed_pair(x, y, c, ws, &pa.side[1].x, &pa.side[1].y, &ra);
    pa.side[1].stop = 0;
    pa.side[0].x = to_dev(x);
    pa.side[0].y = to_dev(y);
    pa.side[0].stop = c;
    if (sizing) return TTC_OK;
    if (ws.off > ws_bytes) return fail(TTC_ERR_WORKSPACE, "workspace too small");
    pa.side[0].out = reinterpret_cast<float*>(V);
    pa.side[1].out = reinterpret_cast<float*>(W);
    pa.m16 = m16;
    TTC_HIP(launch_core_reverse(ra, s));
    TTC_HIP(launch_pair_lds(x->dtype, pa, 2, s));
    TTC_HIP(launch_meet(x->dtype, W, V, (int)rp, d_out, s));
    return TTC_OK;
  }
  if (lds_path(x, y)) {
    // one right-to-left sweep with the interface in LDS, then the first cores
    if (sizing) return TTC_OK;
    PairLdsArgs pa;
    std::memset(&pa, 0, sizeof(pa));
    pa.side[0].x = to_dev(x);
    pa.side[0].y = to_dev(y);
    pa.side[0].stop = 1;
    pa.side[0].inner = d_out;
    pa.m16 = m16;
    TTC_HIP(launch_pair_lds(x->dtype, pa, 1, s));
    return TTC_OK;
  }
  const int N = x->order, c = N / 2;
  const size_t cs = comp_size(x->dtype);
  const size_t rp = (size_t)x->ranks[c] * y->ranks[c];
  void* W = ws.take(rp * cs);
  void* V = ws.take(rp * cs);
  SweepSizing sz;
  TTC_TRY(size_sweep(x, y, 0, N, &sz));
  void* tg = sz.t_global ? ws.take(2 * sz.t_block_bytes) : nullptr;
  void* ig = sz.i_global ? ws.take(2 * sz.i_block_bytes) : nullptr;
  if (sizing) return TTC_OK;
  if (ws.off > ws_bytes) return fail(TTC_ERR_WORKSPACE, "workspace too small");
  SweepArgs a;
  std::memset(&a, 0, sizeof(a));
  a.x = to_dev(x);
  a.y = to_dev(y);
  a.dir[0] = 0;
  a.dir[1] = 1;
  a.stop[0] = c;
  a.stop[1] = c;
  a.out[0] = W;
  a.out[1] = V;
  a.max_rp = sz.max_rp;
  a.tcap = sz.tcap;
  a.t_global = tg;
  a.t_stride = sz.tcap;
  a.i_global = ig;
  a.i_stride = 2L * sz.max_rp;
  a.chain = sz.chain;
  TTC_HIP(launch_sweep(x->dtype, a, 2, sz.lds, s));
  TTC_HIP(launch_meet(x->dtype, W, V, (int)rp, d_out, s));
  return TTC_OK;
}

// Precision of an inner product: AUTO, the precision AUTO picks, or BF16
// for BF16 cores on the LDS path (every rank <= 128): the BF16-MFMA steps.
ttc_status check_inner_prec(const ttc_tt* x, const ttc_tt* y, ttc_prec prec) {
  if (prec != TTC_PREC_BF16) return check_prec(prec, x->dtype);
  if (x->dtype != TTC_BF16) return fail(TTC_ERR_UNSUPPORTED, "BF16 precision needs BF16 cores");
  if (!lds_path(x, y)) return fail(TTC_ERR_UNSUPPORTED, "BF16 MFMA steps need every rank <= 128");
  return TTC_OK;
}

ttc_status check_out_tt(const ttc_tt* o, const std::vector<int>& modes, const std::vector<int>& ranks,
                        ttc_dtype want) {
  if (!o) return fail(TTC_ERR_NULL, "output TT is NULL");
  if (o->order != (int)modes.size()) return fail(TTC_ERR_SHAPE, "output TT has the wrong order");
  if (!o->modes || !o->ranks || !o->cores) return fail(TTC_ERR_NULL, "output TT: NULL descriptor array");
  if (o->dtype != want) return fail(TTC_ERR_DTYPE, "output TT has the wrong dtype");
  for (size_t k = 0; k < modes.size(); ++k) {
    if (o->modes[k] != modes[k]) return fail(TTC_ERR_SHAPE, "output TT mode " + std::to_string(k) + " mismatch");
    if (!o->cores[k]) return fail(TTC_ERR_NULL, "output TT: NULL core pointer");
  }
  for (size_t k = 0; k < ranks.size(); ++k)
    if (o->ranks[k] != ranks[k]) return fail(TTC_ERR_RANK, "output TT rank " + std::to_string(k) + " mismatch");
  return TTC_OK;
}

// Fill the lift description for a natural-order TT.
void build_lift(const ttc_tt* x, const ttc_tt* y, BlockKind kind, int k, const void* K, void* const* out_cores,
                LiftArgs* la, int* total_lines) {
  std::memset(la, 0, sizeof(*la));
  const int N = x->order;
  const int Q = y->ranks[k];
  la->Q = Q;
  la->kr = x->ranks[k];
  la->K = K;
  int nc = 0, lines = 0;
  auto add = [&](int op, int r0, int n, int r1, int d0, int d1, const void* src) {
    LiftCore& c = la->c[nc];
    c.op = op;
    c.r0 = r0;
    c.n = n;
    c.r1 = r1;
    c.d0 = d0;
    c.d1 = d1;
    c.src = src;
    c.dst = out_cores[nc];
    lines += d0 * n;
    ++nc;
  };
  if (kind == BK_PREFIX) {
    for (int m = k; m < N; ++m) {
      const int r0 = x->ranks[m], r1 = x->ranks[m + 1];
      if (m == k)
        add(LIFT_ABSORB_L, r0, x->modes[m], r1, 1, r1 * Q, x->cores[m]);
      else
        add(LIFT_DELTA, r0, x->modes[m], r1, r0 * Q, r1 * Q, x->cores[m]);
    }
    for (int m = k; m < N; ++m)
      add(LIFT_COPY, y->ranks[m], y->modes[m], y->ranks[m + 1], y->ranks[m], y->ranks[m + 1], y->cores[m]);
  } else {
    for (int m = 0; m < k - 1; ++m)
      add(LIFT_COPY, x->ranks[m], x->modes[m], x->ranks[m + 1], x->ranks[m], x->ranks[m + 1], x->cores[m]);
    add(LIFT_ABSORB_R, x->ranks[k - 1], x->modes[k - 1], x->ranks[k], x->ranks[k - 1], Q, x->cores[k - 1]);
    for (int m = 0; m < k; ++m) {
      const int p0 = y->ranks[m], p1 = y->ranks[m + 1];
      if (m == k - 1)
        add(LIFT_DELTA_LAST, p0, y->modes[m], p1, p0 * Q, 1, y->cores[m]);
      else
        add(LIFT_DELTA, p0, y->modes[m], p1, p0 * Q, p1 * Q, y->cores[m]);
    }
  }
  la->ncores = nc;
  *total_lines = lines;
}

int default_stride(int N) {
  int c = (int)std::ceil(std::sqrt((double)N));
  return c < 1 ? 1 : c;
}

}  // namespace

// =========================================================================
// C ABI
// =========================================================================
extern "C" {

const char* ttc_last_error(void) { return g_err.c_str(); }
const char* ttc_version(void) { return "ttc 0.1 (gfx950)"; }
int32_t ttc_abi_version(void) { return TTC_ABI_VERSION; }

ttc_status tt_contract_inner_query(const ttc_tt* x, const ttc_tt* y, ttc_prec prec, size_t* ws_bytes) {
  TTC_TRY(check_pair(x, y));
  TTC_TRY(check_inner_prec(x, y, prec));
  if (!ws_bytes) return fail(TTC_ERR_NULL, "ws_bytes is NULL");
  Arena a(nullptr);
  TTC_TRY(run_inner(x, y, nullptr, a, 0, true, 0));
  *ws_bytes = a.off;
  return TTC_OK;
}

ttc_status tt_contract_inner(const ttc_tt* x, const ttc_tt* y, ttc_prec prec, double* d_out, void* d_ws,
                             size_t ws_bytes, void* stream) {
  TTC_TRY(check_pair(x, y));
  TTC_TRY(check_inner_prec(x, y, prec));
  if (!d_out) return fail(TTC_ERR_NULL, "d_out is NULL");
  size_t need = 0;
  TTC_TRY(tt_contract_inner_query(x, y, prec, &need));
  if (need > ws_bytes) return fail(TTC_ERR_WORKSPACE, "workspace smaller than tt_contract_inner_query size");
  if (need && !d_ws) return fail(TTC_ERR_NULL, "d_ws is NULL");
  TTC_TRY(ensure_init());
  Arena a(d_ws);
  return run_inner(x, y, d_out, a, ws_bytes, false, (hipStream_t)stream, prec == TTC_PREC_BF16);
}

ttc_status tt_contract_modes_query(const ttc_tt* x, const ttc_tt* y, const int32_t* modes, int32_t n_modes,
                                   ttc_form form, ttc_prec prec, int32_t* out_order, int32_t* out_modes,
                                   int32_t* out_ranks, int64_t* out_elems, size_t* ws_bytes) {
  TTC_TRY(check_pair(x, y));
  TTC_TRY(check_inner_prec(x, y, prec));
  BlockKind kind;
  int k;
  TTC_TRY(classify(x->order, modes, n_modes, &kind, &k));
  if (form != TTC_JUNCTION && form != TTC_NATURAL_TT && form != TTC_DENSE)
    return fail(TTC_ERR_UNSUPPORTED, "unknown form");
  if (kind == BK_OTHER) return fail(TTC_ERR_UNSUPPORTED, "GPU path needs a prefix, suffix or all positions");
  const size_t cs = comp_size(x->dtype);
  Arena a(nullptr);
  int order = 0;
  int64_t elems = 1;
  std::vector<int> nm, nr;
  if (kind == BK_ALL) {
    TTC_TRY(run_inner(x, y, nullptr, a, 0, true, 0));
    order = 0;
  } else {
    natural_shape(x, y, kind, k, &nm, &nr);
    if (form == TTC_JUNCTION) {
      TTC_TRY(run_junction(x, y, kind, k, nullptr, a, 0, true, 0));
      order = 2;
      elems = (int64_t)x->ranks[k] * y->ranks[k];
      if (out_ranks) {
        out_ranks[0] = x->ranks[k];
        out_ranks[1] = y->ranks[k];
      }
    } else {
      a.take((size_t)x->ranks[k] * y->ranks[k] * cs);  // K
      TTC_TRY(run_junction(x, y, kind, k, nullptr, a, 0, true, 0));
      order = (int)nm.size();
      if (form == TTC_NATURAL_TT) {
        elems = 0;
        for (int m = 0; m < order; ++m) elems += (int64_t)nr[m] * nm[m] * nr[m + 1];
      } else {
        elems = 1;
        for (int m = 0; m < order; ++m) elems *= nm[m];
        for (int m = 0; m < order; ++m) a.take((size_t)nr[m] * nm[m] * nr[m + 1] * cs);
      }
      if (out_modes)
        for (int m = 0; m < order; ++m) out_modes[m] = nm[m];
      if (out_ranks)
        for (int m = 0; m <= order; ++m) out_ranks[m] = nr[m];
    }
  }
  if (out_order) *out_order = order;
  if (out_elems) *out_elems = elems;
  if (ws_bytes) *ws_bytes = a.off;
  return TTC_OK;
}

ttc_status tt_contract_modes(const ttc_tt* x, const ttc_tt* y, const int32_t* modes, int32_t n_modes,
                             ttc_form form, ttc_prec prec, void* out_junction, const ttc_tt* out_tt,
                             void* out_dense, double* out_scalar, void* d_ws, size_t ws_bytes, void* stream) {
  size_t need = 0;
  int32_t order = 0;
  int64_t elems = 0;
  TTC_TRY(tt_contract_modes_query(x, y, modes, n_modes, form, prec, &order, nullptr, nullptr, &elems, &need));
  const bool m16 = prec == TTC_PREC_BF16;
  if (need > ws_bytes) return fail(TTC_ERR_WORKSPACE, "workspace smaller than tt_contract_modes_query size");
  if (need && !d_ws) return fail(TTC_ERR_NULL, "d_ws is NULL");
  BlockKind kind;
  int k;
  TTC_TRY(classify(x->order, modes, n_modes, &kind, &k));
  hipStream_t s = (hipStream_t)stream;
  const ttc_dtype cdt = x->dtype == TTC_F64 ? TTC_F64 : TTC_F32;
  const size_t cs = comp_size(x->dtype);
  if (kind == BK_ALL) {
    if (!out_scalar) return fail(TTC_ERR_NULL, "out_scalar is NULL (every position contracted)");
    TTC_TRY(ensure_init());
    Arena a(d_ws);
    return run_inner(x, y, out_scalar, a, ws_bytes, false, s, m16);
  }
  std::vector<int> nm, nr;
  natural_shape(x, y, kind, k, &nm, &nr);
  if (form == TTC_JUNCTION) {
    if (!out_junction) return fail(TTC_ERR_NULL, "out_junction is NULL");
    TTC_TRY(ensure_init());
    Arena a(d_ws);
    return run_junction(x, y, kind, k, out_junction, a, ws_bytes, false, s, m16);
  }
  if (form == TTC_NATURAL_TT) TTC_TRY(check_out_tt(out_tt, nm, nr, cdt));
  if (form == TTC_DENSE) {
    if (!out_dense) return fail(TTC_ERR_NULL, "out_dense is NULL");
    for (int r : nr)
      if (r > 64) return fail(TTC_ERR_UNSUPPORTED, "dense form limited to natural ranks <= 64");
  }
  TTC_TRY(ensure_init());
  Arena a(d_ws);
  void* K = a.take((size_t)x->ranks[k] * y->ranks[k] * cs);
  TTC_TRY(run_junction(x, y, kind, k, K, a, ws_bytes, false, s, m16));
  std::vector<void*> cores(nm.size());
  if (form == TTC_NATURAL_TT) {
    for (size_t m = 0; m < nm.size(); ++m) cores[m] = out_tt->cores[m];
  } else {
    for (size_t m = 0; m < nm.size(); ++m) cores[m] = a.take((size_t)nr[m] * nm[m] * nr[m + 1] * cs);
  }
  LiftArgs la;
  int lines = 0;
  build_lift(x, y, kind, k, K, cores.data(), &la, &lines);
  TTC_HIP(launch_lift(x->dtype, la, lines, s));
  if (form == TTC_DENSE) {
    DenseArgs da;
    std::memset(&da, 0, sizeof(da));
    da.t.order = (int)nm.size();
    for (size_t m = 0; m < nm.size(); ++m) {
      da.t.modes[m] = nm[m];
      da.t.cores[m] = cores[m];
    }
    for (size_t m = 0; m < nr.size(); ++m) da.t.ranks[m] = nr[m];
    da.numel = elems;
    da.out = out_dense;
    TTC_HIP(launch_dense(cdt == TTC_F64, da, s));
  }
  return TTC_OK;
}

ttc_status tt_mode_n_product(const ttc_tt* x, int32_t count, const int32_t* modes, const void* const* d_A,
                             const int32_t* J, const ttc_tt* y, void* stream) {
  TTC_TRY(check_tt(x, "x"));
  if (!y) return fail(TTC_ERR_NULL, "y is NULL");
  if (!modes || !d_A || !J) return fail(TTC_ERR_NULL, "modes, d_A or J is NULL");
  if (count < 1 || count > x->order) return fail(TTC_ERR_MODE, "count outside [1, order]");
  if (y->order != x->order) return fail(TTC_ERR_SHAPE, "y has the wrong order");
  if (!y->modes || !y->ranks || !y->cores) return fail(TTC_ERR_NULL, "y: NULL descriptor array");
  if (y->dtype != x->dtype) return fail(TTC_ERR_DTYPE, "y dtype differs from x");
  std::vector<int> seen(x->order, -1);
  for (int c = 0; c < count; ++c) {
    if (modes[c] < 0 || modes[c] >= x->order) return fail(TTC_ERR_MODE, "mode index out of range");
    if (seen[modes[c]] >= 0) return fail(TTC_ERR_MODE, "repeated mode index");
    seen[modes[c]] = c;
    if (J[c] < 1) return fail(TTC_ERR_SHAPE, "J < 1");
    if (!d_A[c]) return fail(TTC_ERR_NULL, "NULL matrix pointer");
    if (!y->cores[modes[c]]) return fail(TTC_ERR_NULL, "NULL output core");
  }
  for (int k = 0; k <= x->order; ++k)
    if (y->ranks[k] != x->ranks[k]) return fail(TTC_ERR_RANK, "y ranks differ from x");
  for (int k = 0; k < x->order; ++k) {
    const int want = seen[k] >= 0 ? J[seen[k]] : x->modes[k];
    if (y->modes[k] != want) return fail(TTC_ERR_SHAPE, "y mode " + std::to_string(k) + " mismatch");
  }
  ModeNArgs ma;
  std::memset(&ma, 0, sizeof(ma));
  ma.count = count;
  long total = 0;
  for (int c = 0; c < count; ++c) {
    const int k = modes[c];
    ModeNEntry& e = ma.e[c];
    e.r0 = x->ranks[k];
    e.I = x->modes[k];
    e.r1 = x->ranks[k + 1];
    e.J = J[c];
    e.first = total;
    e.src = x->cores[k];
    e.A = d_A[c];
    e.dst = y->cores[k];
    total += (long)e.r0 * e.J * e.r1;
  }
  ma.total = total;
  TTC_HIP(launch_mode_n(x->dtype, ma, (hipStream_t)stream));
  return TTC_OK;
}

ttc_status ttm_apply_query(const ttc_ttm* m, const ttc_tt* v, int32_t* out_ranks, int64_t* out_elems) {
  if (!m) return fail(TTC_ERR_NULL, "m is NULL");
  TTC_TRY(check_tt(v, "v"));
  if (m->order != v->order) return fail(TTC_ERR_SHAPE, "m and v have different orders");
  if (!m->rows || !m->cols || !m->ranks || !m->cores) return fail(TTC_ERR_NULL, "m: NULL descriptor array");
  if (m->dtype != v->dtype) return fail(TTC_ERR_DTYPE, "m and v have different dtypes");
  const int N = m->order;
  if (m->ranks[0] != 1 || m->ranks[N] != 1) return fail(TTC_ERR_RANK, "m: boundary ranks must be 1");
  int64_t elems = 0;
  for (int k = 0; k < N; ++k) {
    if (m->cols[k] != v->modes[k]) return fail(TTC_ERR_SHAPE, "m column modes differ from v modes");
    if (m->rows[k] < 1 || m->ranks[k] < 1) return fail(TTC_ERR_SHAPE, "m: bad shape");
    if (!m->cores[k]) return fail(TTC_ERR_NULL, "m: NULL core pointer");
    const double ne = (double)m->ranks[k] * v->ranks[k] * m->rows[k] * m->ranks[k + 1] * v->ranks[k + 1];
    if (ne >= 2147483647.0) return fail(TTC_ERR_SHAPE, "output core too large");
    elems += (int64_t)m->ranks[k] * v->ranks[k] * m->rows[k] * m->ranks[k + 1] * v->ranks[k + 1];
  }
  if (out_ranks)
    for (int k = 0; k <= N; ++k) out_ranks[k] = m->ranks[k] * v->ranks[k];
  if (out_elems) *out_elems = elems;
  return TTC_OK;
}

ttc_status ttm_apply(const ttc_ttm* m, const ttc_tt* v, ttc_prec prec, const ttc_tt* out, void* stream) {
  TTC_TRY(ttm_apply_query(m, v, nullptr, nullptr));
  const int N = m->order;
  bool bf16_mfma = false;
  if (prec == TTC_PREC_BF16 || prec == TTC_PREC_AUTO) {
    if (v->dtype == TTC_BF16) bf16_mfma = true;
    else if (prec == TTC_PREC_BF16) return fail(TTC_ERR_UNSUPPORTED, "BF16 precision needs BF16 inputs");
  } else {
    TTC_TRY(check_prec(prec, v->dtype));
  }
  std::vector<int> om(m->rows, m->rows + N), orr(N + 1);
  for (int k = 0; k <= N; ++k) orr[k] = m->ranks[k] * v->ranks[k];
  TTC_TRY(check_out_tt(out, om, orr, v->dtype == TTC_F64 ? TTC_F64 : TTC_F32));
  MpoArgs a;
  std::memset(&a, 0, sizeof(a));
  a.ncores = N;
  for (int k = 0; k < N; ++k) {
    MpoCore& c = a.c[k];
    c.a0 = m->ranks[k];
    c.I = m->rows[k];
    c.J = m->cols[k];
    c.a1 = m->ranks[k + 1];
    c.r0 = v->ranks[k];
    c.r1 = v->ranks[k + 1];
    c.w = m->cores[k];
    c.v = v->cores[k];
    c.out = out->cores[k];
  }
  TTC_HIP(launch_mpo(v->dtype, bf16_mfma, a, (hipStream_t)stream));
  return TTC_OK;
}

}  // extern "C"

namespace {
// Launch shape of the per-slice gradient kernel: one block per (X or Y,
// core, mode index) and a product buffer of max_k R_k x P_{k+1} elements,
// in LDS when it fits.
struct GradCoreShape {
  int blocks;
  long elems;
  bool global;
};
GradCoreShape grad_core_shape(const ttc_tt* x, const ttc_tt* y, size_t cs) {
  int imax = 1;
  long e = 1;
  for (int k = 0; k < x->order; ++k) {
    imax = std::max(imax, x->modes[k]);
    e = std::max(e, (long)x->ranks[k] * y->ranks[k + 1]);
  }
  GradCoreShape g;
  g.blocks = 2 * x->order * imax;
  g.elems = e;
  g.global = (size_t)e * cs > (size_t)(lds_limit_bytes() - 1024);
  return g;
}

// Buffers of the gradient's LDS-sweep path: every V_{k+1} and W_k stored
// (slot k of segV / segW, R x P row-major FP32), the reversed pair for the
// left-to-right sweep, and the product buffers of the slice kernel.
struct GradLds {
  int max_rp = 1;
  float* segV = nullptr;
  float* segW = nullptr;
  TTDev xr, yr;
  CoreRevArgs ra;
  GradCoreShape gc;
  void* g_global = nullptr;
};
void grad_lds_take(const ttc_tt* x, const ttc_tt* y, Arena& a, GradLds* g) {
  const int N = x->order;
  long m = 1;
  for (int b = 0; b <= N; ++b) m = std::max(m, (long)x->ranks[b] * y->ranks[b]);
  g->max_rp = (int)m;
  g->segV = reinterpret_cast<float*>(a.take((size_t)N * m * sizeof(float)));
  g->segW = reinterpret_cast<float*>(a.take((size_t)N * m * sizeof(float)));
  reversed_pair(x, y, N, a, &g->xr, &g->yr, &g->ra);
  g->gc = grad_core_shape(x, y, sizeof(float));
  g->g_global = g->gc.global ? a.take((size_t)g->gc.blocks * g->gc.elems * sizeof(float)) : nullptr;
}
// The gradient stores every interface (LDS-resident sweeps) when the pair
// takes the LDS path and the caller asked for no checkpoint stride; a
// positive stride always selects checkpointing with recomputation.
bool grad_stores_all(const ttc_tt* x, const ttc_tt* y, int32_t ckpt_stride) {
  return ckpt_stride <= 0 && lds_path(x, y);
}
}  // namespace

extern "C" {

ttc_status tt_contract_inner_bwd_query(const ttc_tt* x, const ttc_tt* y, int32_t ckpt_stride, size_t* ws_bytes) {
  TTC_TRY(check_pair(x, y));
  if (!ws_bytes) return fail(TTC_ERR_NULL, "ws_bytes is NULL");
  if (grad_stores_all(x, y, ckpt_stride)) {
    Arena a(nullptr);
    GradLds g;
    grad_lds_take(x, y, a, &g);
    *ws_bytes = a.off;
    return TTC_OK;
  }
  const int N = x->order;
  const int c = ckpt_stride > 0 ? std::min<int>(ckpt_stride, N) : default_stride(N);
  const int ns = (N + c - 1) / c;
  SweepSizing sz;
  TTC_TRY(size_sweep(x, y, 0, N, &sz, false));
  const size_t cs = comp_size(x->dtype);
  Arena a(nullptr);
  a.take((size_t)ns * sz.max_rp * cs);
  a.take((size_t)ns * sz.max_rp * cs);
  a.take((size_t)ns * c * sz.max_rp * cs);
  a.take((size_t)ns * c * sz.max_rp * cs);
  if (sz.t_global) a.take((size_t)std::max(ns, 2) * sz.t_block_bytes);
  if (sz.i_global) a.take((size_t)std::max(ns, 2) * sz.i_block_bytes);
  const GradCoreShape gc = grad_core_shape(x, y, cs);
  if (gc.global) a.take((size_t)gc.blocks * gc.elems * cs);
  *ws_bytes = a.off;
  return TTC_OK;
}

ttc_status tt_contract_inner_bwd(const ttc_tt* x, const ttc_tt* y, const double* d_gz, void* const* d_dx,
                                 void* const* d_dy, int32_t ckpt_stride, void* d_ws, size_t ws_bytes,
                                 void* stream) {
  size_t need = 0;
  TTC_TRY(tt_contract_inner_bwd_query(x, y, ckpt_stride, &need));
  if (!d_gz) return fail(TTC_ERR_NULL, "d_gz is NULL");
  if (need > ws_bytes) return fail(TTC_ERR_WORKSPACE, "workspace smaller than tt_contract_inner_bwd_query size");
  if (need && !d_ws) return fail(TTC_ERR_NULL, "d_ws is NULL");
  const int N = x->order;
  for (int k = 0; k < N; ++k) {
    if (d_dx && !d_dx[k]) return fail(TTC_ERR_NULL, "NULL gradient buffer in d_dx");
    if (d_dy && !d_dy[k]) return fail(TTC_ERR_NULL, "NULL gradient buffer in d_dy");
  }
  TTC_TRY(ensure_init());
  hipStream_t s = (hipStream_t)stream;
  if (grad_stores_all(x, y, ckpt_stride)) {
    // two workgroups store every interface (V right to left, W as the
    // reversed pair's V), then one wide launch forms every slice
    Arena a(d_ws);
    GradLds gl;
    grad_lds_take(x, y, a, &gl);
    TTC_HIP(launch_core_reverse(gl.ra, s));
    PairLdsArgs pa;
    std::memset(&pa, 0, sizeof(pa));
    pa.side[0].x = to_dev(x);
    pa.side[0].y = to_dev(y);
    pa.side[0].stop = 1;
    pa.side[0].all = gl.segV;  // V_k in slot k - 1
    pa.side[0].slot_a = 1;
    pa.side[0].slot_b = -1;
    pa.side[0].all_stride = gl.max_rp;
    pa.side[1].x = gl.xr;
    pa.side[1].y = gl.yr;
    pa.side[1].stop = 1;
    pa.side[1].all = gl.segW;  // V'_j = W_{N-j} in slot N - j
    pa.side[1].slot_a = -1;
    pa.side[1].slot_b = N;
    pa.side[1].all_stride = gl.max_rp;
    TTC_HIP(launch_pair_lds(x->dtype, pa, 2, s));
    GradArgs g;
    std::memset(&g, 0, sizeof(g));
    g.x = to_dev(x);
    g.y = to_dev(y);
    g.segV = gl.segV;
    g.segW = gl.segW;
    g.max_rp = gl.max_rp;
    g.g_global = gl.g_global;
    g.g_stride = gl.gc.elems;
    g.gz = d_gz;
    for (int k = 0; k < N; ++k) {
      g.dx[k] = d_dx ? d_dx[k] : nullptr;
      g.dy[k] = d_dy ? d_dy[k] : nullptr;
    }
    TTC_HIP(launch_grad_core(x->dtype, g, gl.gc.blocks, gl.gc.global ? 0 : (size_t)gl.gc.elems * sizeof(float), s));
    return TTC_OK;
  }
  const int c = ckpt_stride > 0 ? std::min<int>(ckpt_stride, N) : default_stride(N);
  const int ns = (N + c - 1) / c;
  SweepSizing sz;
  TTC_TRY(size_sweep(x, y, 0, N, &sz, false));
  const size_t cs = comp_size(x->dtype);
  Arena a(d_ws);
  GradArgs g;
  std::memset(&g, 0, sizeof(g));
  g.x = to_dev(x);
  g.y = to_dev(y);
  g.stride = c;
  g.nseg = ns;
  g.ckW = a.take((size_t)ns * sz.max_rp * cs);
  g.ckV = a.take((size_t)ns * sz.max_rp * cs);
  g.segV = a.take((size_t)ns * c * sz.max_rp * cs);
  g.segW = a.take((size_t)ns * c * sz.max_rp * cs);
  g.t_global = sz.t_global ? a.take((size_t)std::max(ns, 2) * sz.t_block_bytes) : nullptr;
  g.t_stride = sz.tcap;
  g.i_global = sz.i_global ? a.take((size_t)std::max(ns, 2) * sz.i_block_bytes) : nullptr;
  g.i_stride = 2L * sz.max_rp;
  const GradCoreShape gc = grad_core_shape(x, y, cs);
  g.g_global = gc.global ? a.take((size_t)gc.blocks * gc.elems * cs) : nullptr;
  g.g_stride = gc.elems;
  g.gz = d_gz;
  g.max_rp = sz.max_rp;
  g.tcap = sz.tcap;
  for (int k = 0; k < N; ++k) {
    g.dx[k] = d_dx ? d_dx[k] : nullptr;
    g.dy[k] = d_dy ? d_dy[k] : nullptr;
  }
  TTC_HIP(launch_grad_ckpt(x->dtype, g, sz.lds, s));
  TTC_HIP(launch_grad_seg(x->dtype, g, sz.lds, s));
  TTC_HIP(launch_grad_core(x->dtype, g, gc.blocks, gc.global ? 0 : (size_t)gc.elems * cs, s));
  return TTC_OK;
}

}  // extern "C"
