// Host side of the TT layer: TT-matrix x dense batch (forward, backward)
// and the MSE loss.  See layer.hip for the schedule.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "ttc_layer.h"

namespace ttc {
ttc_status fail(ttc_status s, const std::string& msg);
}
using namespace ttc;

#define TTC_TRY(expr)            \
  do {                           \
    ttc_status _s = (expr);      \
    if (_s != TTC_OK) return _s; \
  } while (0)
#define TTC_HIP(expr)                                                                                    \
  do {                                                                                                   \
    hipError_t _e = (expr);                                                                              \
    if (_e != hipSuccess) return fail(TTC_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)

namespace {

struct Arena {
  char* base;
  size_t off = 0;
  explicit Arena(void* b) : base((char*)b) {}
  float* take(size_t elems) {
    off = (off + 255) & ~(size_t)255;
    float* p = base ? reinterpret_cast<float*>(base + off) : nullptr;
    off += elems * sizeof(float);
    return p;
  }
};

const size_t kSlabElems = (size_t)8 << 20;  // split-K partial slabs (32 MB)

ttc_status check_ttm(const ttc_ttm* m) {
  if (!m) return fail(TTC_ERR_NULL, "m is NULL");
  if (m->order < 1 || m->order > TTC_MAX_ORDER) return fail(TTC_ERR_SHAPE, "m: order outside [1, 32]");
  if (!m->rows || !m->cols || !m->ranks || !m->cores) return fail(TTC_ERR_NULL, "m: NULL descriptor array");
  if (m->dtype != TTC_F32) return fail(TTC_ERR_DTYPE, "TT layer cores must be FP32");
  const int d = m->order;
  if (m->ranks[0] != 1 || m->ranks[d] != 1) return fail(TTC_ERR_RANK, "m: boundary ranks must be 1");
  double rows = 1, cols = 1;
  for (int k = 0; k < d; ++k) {
    if (m->rows[k] < 1 || m->cols[k] < 1) return fail(TTC_ERR_SHAPE, "m: mode size < 1");
    if (m->ranks[k] < 1) return fail(TTC_ERR_RANK, "m: rank < 1");
    if (!m->cores[k]) return fail(TTC_ERR_NULL, "m: NULL core pointer");
    rows *= m->rows[k];
    cols *= m->cols[k];
  }
  if (rows * cols >= 2147483647.0) return fail(TTC_ERR_SHAPE, "dense matrix larger than 2^31 entries");
  return TTC_OK;
}

// Buffers of one call, carved from the workspace in a fixed order.
struct LayerPlan {
  int d;
  long rows, cols;                 // prod I, prod J
  std::vector<long> mprefix;       // |m_<k| for k = 0..d
  std::vector<float*> L;           // L_k, k = 1..d-1 (L_1 aliases core 0)
  float* Dp = nullptr;             // pair-mode order buffer (prod I J)
  float* Wd = nullptr;             // dense matrix / its gradient
  float* RA = nullptr;             // right-environment ping-pong
  float* RB = nullptr;
  float* slab = nullptr;
  // BF16 operand copies for the 256 x 256-tile BF16 products (when used)
  uint16_t* A16 = nullptr;         // X or dY, k contiguous
  uint16_t* B16 = nullptr;         // W or W^T
  uint16_t* C16 = nullptr;         // dY^T
  uint16_t* D16 = nullptr;         // X^T
};

// A product goes to the BF16 tile kernel when its reduction length is a
// multiple of 8 and it has enough 256 x 256 tiles to fill the GPU.
// TTC_GEMM16=0 keeps every BF16 product on the 128 x 128-tile kernel (for
// timing the two against each other).
bool use_gemm16(long M, long N, long K) {
  static const bool off = [] {
    const char* e = std::getenv("TTC_GEMM16");
    return e && e[0] == '0';
  }();
  return !off && K % 8 == 0 && ((M + 255) / 256) * ((N + 255) / 256) >= 64;
}

void plan_layer(const ttc_ttm* m, bool backward, bool bf16, long batch, Arena& a, LayerPlan* p) {
  const int d = m->order;
  p->d = d;
  p->rows = 1;
  p->cols = 1;
  for (int k = 0; k < d; ++k) {
    p->rows *= m->rows[k];
    p->cols *= m->cols[k];
  }
  p->mprefix.assign(d + 1, 1);
  for (int k = 0; k < d; ++k) p->mprefix[k + 1] = p->mprefix[k] * (long)m->rows[k] * m->cols[k];
  p->L.assign(d + 1, nullptr);
  p->L[1] = reinterpret_cast<float*>(m->cores[0]);
  for (int k = 2; k < d; ++k) p->L[k] = a.take((size_t)p->mprefix[k] * m->ranks[k]);
  p->Dp = a.take((size_t)p->mprefix[d]);
  p->Wd = a.take((size_t)p->rows * p->cols);
  if (backward) {
    long mx = 1;
    for (int k = 1; k < d; ++k) mx = std::max(mx, p->mprefix[k] * (long)m->ranks[k]);
    p->RA = a.take((size_t)mx);
    p->RB = a.take((size_t)mx);
  }
  p->slab = a.take(kSlabElems);
  if (bf16) {
    auto take16 = [&](long n) { return reinterpret_cast<uint16_t*>(a.take((size_t)(n + 1) / 2)); };
    const bool fwd16 = use_gemm16(batch, p->rows, p->cols);
    const bool dx16 = backward && use_gemm16(batch, p->cols, p->rows);
    const bool dw16 = backward && use_gemm16(p->rows, p->cols, batch);
    if (fwd16 || dx16) {
      p->A16 = take16(batch * std::max(p->rows, p->cols));
      p->B16 = take16(p->rows * p->cols);
    }
    if (dw16) {
      p->C16 = take16(p->rows * batch);
      p->D16 = take16(p->cols * batch);
    }
  }
}

// C (M x N, ldc) = A . B^T on BF16 operands with k contiguous.
ttc_status gemm16(const uint16_t* A, long lda, const uint16_t* B, long ldb, float* C, long ldc, int M, int N, int K,
                  hipStream_t s) {
  static std::atomic<bool> done[kMaxDevices];
  TTC_HIP(once_per_device(done, [] { return gemm16_set_lds(); }));
  Gemm16Args g;
  std::memset(&g, 0, sizeof(g));
  g.M = M;
  g.N = N;
  g.K = K;
  g.lda = lda;
  g.ldb = ldb;
  g.ldc = ldc;
  g.A = A;
  g.B = B;
  g.C = C;
  g.alpha = 1.f;
  g.splits = 1;
  const int tiles = ((M + 255) / 256) * ((N + 255) / 256);
  g.per_xcd = (tiles % 8 == 0) ? tiles / 8 : 0;
  TTC_HIP(launch_gemm16(g, s));
  return TTC_OK;
}

bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

// One GEMM with split-K chosen to give the GPU enough workgroups.
ttc_status gemm(bool a_kc, const float* A, long lda, bool b_kc, const float* B, long ldb, float* C, long ldc, int M,
                int N, int K, bool bf16, float* slab, hipStream_t s, const IdxMap* map = nullptr,
                size_t slab_elems = kSlabElems) {
  GemmArgs g;
  std::memset(&g, 0, sizeof(g));
  if (map) {
    g.mapped = true;
    g.map = *map;
  }
  g.M = M;
  g.N = N;
  g.K = K;
  g.lda = lda;
  g.ldb = ldb;
  g.ldc = ldc;
  g.A = A;
  g.B = B;
  g.C = C;
  g.alpha = 1.f;
  g.vec_a = (lda % 4 == 0) && aligned16(A);
  g.vec_b = (ldb % 4 == 0) && aligned16(B);
  g.tile = gemm_tile(M, N);
  int tm = 128, tn = 128;
  gemm_tile_dims(g.tile, &tm, &tn);
  const long tiles = (long)((M + tm - 1) / tm) * ((N + tn - 1) / tn);
  const int bk = gemm_bk(bf16);
  int splits = 1;
  if (tiles < 512 && !map && slab) {
    // about 1024 workgroups; at most 256 partial slabs (the reduction reads
    // every slab once per output element), 1024 for outputs of at most 64 K
    // elements
    const long cap = (long)M * N <= 65536 ? 1024L : 256L;
    long want = std::min(cap, (1024 + tiles - 1) / tiles);
    long by_k = K / (4L * bk);
    long by_slab = (long)(slab_elems / ((size_t)M * N));
    splits = (int)std::max(1L, std::min(want, std::min(by_k, by_slab)));
  }
  g.splits = splits;
  g.slab = slab;
  TTC_HIP(launch_gemm(a_kc, b_kc, bf16, g, s));
  return TTC_OK;
}

// The pair-mode <-> matrix permutation of an MPO's dense matrix: the tiled
// kernel when a tile of at least two leading matrix digits fits in LDS,
// else one thread per element.  trans: the matrix is W^T (cols x rows);
// dst16 (dir 0): written as BF16.  The per-element kernel serves only the
// FP32 untransposed form: *done is false when it would be needed for the
// others.
ttc_status permute_dense(const ttc_ttm* m, int dir, const float* src, float* dst, hipStream_t s,
                         bool trans = false, uint16_t* dst16 = nullptr, bool* done = nullptr) {
  const int d = m->order;
  std::vector<long> pstride(d), ri(d), cj(d);
  pstride[d - 1] = 1;
  for (int k = d - 2; k >= 0; --k) pstride[k] = pstride[k + 1] * m->rows[k + 1] * m->cols[k + 1];
  ri[0] = cj[0] = 1;
  for (int k = 1; k < d; ++k) {
    ri[k] = ri[k - 1] * m->rows[k - 1];
    cj[k] = cj[k - 1] * m->cols[k - 1];
  }
  const long rows = ri[d - 1] * m->rows[d - 1], cols = cj[d - 1] * m->cols[d - 1];
  // matrix strides of the digits i_k and j_k; pair-mode strides
  std::vector<long> si(d), sj(d), pi(d), pj(d);
  for (int k = 0; k < d; ++k) {
    si[k] = trans ? ri[k] : ri[k] * cols;
    sj[k] = trans ? cj[k] * rows : cj[k];
    pi[k] = (long)m->cols[k] * pstride[k];
    pj[k] = pstride[k];
  }
  // the matrix's contiguous digits: j_0, j_1, .. (W) or i_0, i_1, .. (W^T)
  const int* lrad = trans ? m->rows : m->cols;
  const std::vector<long>& lP = trans ? pi : pj;
  const std::vector<long>& lM = trans ? si : sj;
  const int* orad_other = trans ? m->cols : m->rows;
  const std::vector<long>& oP = trans ? pj : pi;
  const std::vector<long>& oM = trans ? sj : si;
  long total = rows * cols;
  if (done) *done = true;
  if (d >= 2) {
    const int Bp = m->rows[d - 1] * m->cols[d - 1];
    int t = 0, Bm = 1;
    while (t < d - 1 && (long)Bm * lrad[t] <= 256 && (long)Bm * lrad[t] * (Bp + 1) <= kTilePermElems + 64) {
      Bm *= lrad[t];
      ++t;
    }
    if (Bm >= 2) {
      TilePermArgs tp;
      std::memset(&tp, 0, sizeof(tp));
      tp.dir = dir;
      tp.Bp = Bp;
      tp.Jl = m->cols[d - 1];
      tp.sMi = si[d - 1];
      tp.sMj = sj[d - 1];
      tp.t = t;
      tp.Bm = Bm;
      for (int k = 0; k < t; ++k) {
        tp.jrad[k] = lrad[k];
        tp.sPj[k] = lP[k];
      }
      // outer digits, the matrix's faster ones first
      int q = 0;
      for (int k = t; k < d - 1; ++k, ++q) {
        tp.orad[q] = lrad[k];
        tp.osP[q] = lP[k];
        tp.osM[q] = lM[k];
      }
      for (int k = 0; k < d - 1; ++k, ++q) {
        tp.orad[q] = orad_other[k];
        tp.osP[q] = oP[k];
        tp.osM[q] = oM[k];
      }
      tp.nout = q;
      tp.tiles = total / ((long)Bp * Bm);
      tp.src = src;
      tp.dst = dst;
      tp.dst16 = dir == 0 ? dst16 : nullptr;
      const uintptr_t al = (uintptr_t)src | (dst16 ? 0 : (uintptr_t)dst);
      tp.vec = Bp % 4 == 0 && Bm % 4 == 0 && (al & 15) == 0 && ((uintptr_t)dst16 & 7) == 0;
      TTC_HIP(launch_tile_permute(tp, s));
      return TTC_OK;
    }
  }
  if (trans || dst16) {
    if (done) *done = false;
    return TTC_OK;
  }
  PermArgs pa;
  std::memset(&pa, 0, sizeof(pa));
  pa.dir = dir;
  pa.d = d;
  for (int k = 0; k < d; ++k) {
    pa.I[k] = m->rows[k];
    pa.J[k] = m->cols[k];
    pa.pstride[k] = pstride[k];
  }
  pa.cols = cols;
  pa.total = total;
  pa.src = src;
  pa.dst = dst;
  TTC_HIP(launch_permute(pa, s));
  return TTC_OK;
}

// The chain L_{k+1} = L_k . W^(k) (pair-mode order in Dp).  Keeps every L_k
// in the plan.
ttc_status build_chain(const ttc_ttm* m, LayerPlan& p, hipStream_t s) {
  const int d = m->order;
  const float* cur = reinterpret_cast<const float*>(m->cores[0]);  // L_1: |m_<1| x R_1
  for (int k = 1; k < d; ++k) {
    const long Mk = (long)m->rows[k] * m->cols[k];
    const int R = m->ranks[k], R1 = m->ranks[k + 1];
    float* out = (k + 1 < d) ? p.L[k + 1] : p.Dp;
    TTC_TRY(gemm(true, cur, R, false, reinterpret_cast<const float*>(m->cores[k]), Mk * R1, out, Mk * R1,
                 (int)p.mprefix[k], (int)(Mk * R1), R, false, p.slab, s));
    cur = out;
  }
  return TTC_OK;
}

const float* pair_order(const ttc_ttm* m, const LayerPlan& p) {
  return m->order == 1 ? reinterpret_cast<const float*>(m->cores[0]) : p.Dp;
}

// Dense matrix W[i, j] (FP32, in p.Wd) from the cores: the chain, then the
// pair-mode -> matrix permutation.
ttc_status build_dense(const ttc_ttm* m, LayerPlan& p, hipStream_t s) {
  TTC_TRY(build_chain(m, p, s));
  return permute_dense(m, 0, pair_order(m, p), p.Wd, s);
}

// The BF16 operand of a product with W into p.B16: W (k = j contiguous) or,
// trans, W^T (k = i contiguous), written by the permutation itself when the
// tiled form applies, else through the FP32 matrix and a conversion pass.
ttc_status build_dense16(const ttc_ttm* m, LayerPlan& p, bool trans, hipStream_t s) {
  TTC_TRY(build_chain(m, p, s));
  bool done = false;
  TTC_TRY(permute_dense(m, 0, pair_order(m, p), p.Wd, s, trans, p.B16, &done));
  if (done) return TTC_OK;
  TTC_TRY(permute_dense(m, 0, pair_order(m, p), p.Wd, s));
  if (trans)
    TTC_HIP(launch_cvt16_t(p.Wd, p.B16, p.rows, p.cols, s));
  else
    TTC_HIP(launch_cvt16(p.Wd, p.B16, p.rows * p.cols, s));
  return TTC_OK;
}

// ------------------------------------------------- core-by-core schedule
// Step k: Z_{k+1}[(P_k, Q_k), (i_k, r_{k+1})] = Z_k[(P_k, Q_k), (j_k, r_k)] . Wp_k
// with |P_k| = batch * prod_{t>k} J_t, |Q_k| = prod_{t<k} I_t (see layer.hip).
struct CoresPlan {
  int d = 0;
  std::vector<long> P, Q, K, N;  // per step
  std::vector<float*> Wp;        // permuted cores
  std::vector<float*> Z;         // Z_k, k = 1..d-1
  float* dC[2] = {nullptr, nullptr};  // backward: output gradients of two steps
  float* dWp = nullptr;
  float* slab = nullptr;
};

void cores_shape(const ttc_ttm* m, long batch, CoresPlan* p) {
  const int d = m->order;
  p->d = d;
  p->P.assign(d, 0);
  p->Q.assign(d, 0);
  p->K.assign(d, 0);
  p->N.assign(d, 0);
  for (int k = 0; k < d; ++k) {
    long P = batch, Q = 1;
    for (int t = k + 1; t < d; ++t) P *= m->cols[t];
    for (int t = 0; t < k; ++t) Q *= m->rows[t];
    p->P[k] = P;
    p->Q[k] = Q;
    p->K[k] = (long)m->cols[k] * m->ranks[k];
    p->N[k] = (long)m->rows[k] * m->ranks[k + 1];
  }
}

double cores_flops(const CoresPlan& p) {
  double f = 0;
  for (int k = 0; k < p.d; ++k) f += 2.0 * p.P[k] * p.Q[k] * p.K[k] * p.N[k];
  return f;
}

double dense_flops(const ttc_ttm* m, long batch) {
  double rows = 1, cols = 1, chain = 0, pref = 1;
  for (int k = 0; k < m->order; ++k) {
    if (k > 0) chain += 2.0 * pref * m->ranks[k] * m->rows[k] * m->cols[k] * m->ranks[k + 1];
    pref *= (double)m->rows[k] * m->cols[k];
    rows *= m->rows[k];
    cols *= m->cols[k];
  }
  return chain + 2.0 * batch * rows * cols;
}

void plan_cores(const ttc_ttm* m, long batch, bool backward, Arena& a, CoresPlan* p) {
  cores_shape(m, batch, p);
  const int d = p->d;
  p->Wp.assign(d, nullptr);
  for (int k = 0; k < d; ++k) p->Wp[k] = a.take((size_t)p->K[k] * p->N[k]);
  p->Z.assign(d, nullptr);
  long zmax = 1, cmax = 1, wmax = 1;
  for (int k = 1; k < d; ++k) zmax = std::max(zmax, p->P[k] * p->Q[k] * p->K[k]);
  for (int k = 0; k < d; ++k) {
    cmax = std::max(cmax, p->P[k] * p->Q[k] * p->N[k]);
    wmax = std::max(wmax, p->K[k] * p->N[k]);
  }
  (void)zmax;
  if (backward) {
    // every Z_k kept (the backward reads them), then the gradient buffers
    for (int k = 1; k < d; ++k) p->Z[k] = a.take((size_t)p->P[k] * p->Q[k] * p->K[k]);
    p->dC[0] = a.take((size_t)cmax);
    p->dC[1] = d > 1 ? a.take((size_t)cmax) : nullptr;
    p->dWp = a.take((size_t)wmax);
  } else if (d > 1) {
    float* buf[2] = {a.take((size_t)zmax), d > 2 ? a.take((size_t)zmax) : nullptr};
    // Z_1, Z_2, ... alternate between the two buffers (one suffices for d = 2)
    for (int k = 1; k < d; ++k) p->Z[k] = buf[(k - 1) & 1];
  }
  p->slab = a.take(kSlabElems);
}

// Store map of step k: its output (m = (p', j_{k+1}, q), n = (i_k, r_{k+1}))
// into [P_{k+1}, (i_k, Q_k), j_{k+1}, r_{k+1}] (the last step: Y[b, i_k, Q_k]).
IdxMap step_map(const ttc_ttm* m, const CoresPlan& p, int k) {
  const long Jn = (k + 1 < p.d) ? m->cols[k + 1] : 1, Rn = m->ranks[k + 1], Q = p.Q[k];
  IdxMap mp;
  mp.mr0 = (int)Q;
  mp.mr1 = (int)Jn;
  mp.ms0 = Jn * Rn;
  mp.ms1 = Rn;
  mp.ms2 = (long)m->rows[k] * Q * Jn * Rn;
  mp.nr0 = (int)Rn;
  mp.ns0 = 1;
  mp.ns1 = Q * Jn * Rn;
  return mp;
}

// The inverse of step k's store map as the store map of the product that
// yields the gradient of Z_{k+1} (rows (p', i_k, q), columns (j_{k+1},
// r_{k+1})): it writes the gradient of step k's output straight into that
// output's own layout [(p', j_{k+1}, q), (i_k, r_{k+1})].
IdxMap step_map_inv(const ttc_ttm* m, const CoresPlan& p, int k) {
  const long Jn = m->cols[k + 1], Rn = m->ranks[k + 1], Q = p.Q[k], I = m->rows[k];
  IdxMap mp;
  mp.mr0 = (int)Q;
  mp.mr1 = (int)I;
  mp.ms0 = I * Rn;
  mp.ms1 = Rn;
  mp.ms2 = Jn * Q * I * Rn;
  mp.nr0 = (int)Rn;
  mp.ns0 = 1;
  mp.ns1 = Q * I * Rn;
  return mp;
}

// Forward steps; with Y null the last step is skipped (backward recompute).
ttc_status cores_forward(const ttc_ttm* m, const CoresPlan& p, const float* X, float* Y, bool bf16, hipStream_t s) {
  const int d = p.d;
  for (int k = 0; k < d; ++k)
    TTC_HIP(launch_core_perm(reinterpret_cast<const float*>(m->cores[k]), p.Wp[k], m->ranks[k], m->rows[k],
                             m->cols[k], m->ranks[k + 1], 0, s));
  const float* cur = X;
  for (int k = 0; k < d; ++k) {
    float* out = (k + 1 < d) ? p.Z[k + 1] : Y;
    if (!out) break;
    const IdxMap mp = step_map(m, p, k);
    TTC_TRY(gemm(true, cur, p.K[k], false, p.Wp[k], p.N[k], out, 0, (int)(p.P[k] * p.Q[k]), (int)p.N[k],
                 (int)p.K[k], bf16, p.slab, s, &mp));
    cur = out;
  }
  return TTC_OK;
}

// saved: Z_k and Wp_k are in the workspace from the forward (schedule
// CORES_SAVED), else they are recomputed.  The gradient of the last step's
// output is gathered from dY; every other step's comes from the product
// dZ_{k+1} = dC_{k+1} Wp_{k+1}^T, stored through the inverse map straight
// into the layout of dC_k.
ttc_status cores_backward(const ttc_ttm* m, const CoresPlan& p, const float* X, const float* dY, float* dX,
                          void* const* dcores, bool bf16, bool saved, hipStream_t s) {
  const int d = p.d;
  if (!saved) TTC_TRY(cores_forward(m, p, X, nullptr, bf16, s));
  {
    GatherArgs ga;
    ga.M = p.P[d - 1] * p.Q[d - 1];
    ga.N = p.N[d - 1];
    ga.map = step_map(m, p, d - 1);
    ga.src = dY;
    ga.dst = p.dC[(d - 1) & 1];
    TTC_HIP(launch_gather(ga, s));
  }
  for (int k = d - 1; k >= 0; --k) {
    const long M = p.P[k] * p.Q[k];
    const float* dC = p.dC[k & 1];
    if (dcores) {
      // dWp_k = Z_k^T dC_k: A(m = (j, r), k = row) = Z_k[row * K + m], B(k = row, n) = dC[row * N + n]
      const float* Zk = k == 0 ? X : p.Z[k];
      TTC_TRY(gemm(false, Zk, p.K[k], false, dC, p.N[k], p.dWp, p.N[k], (int)p.K[k], (int)p.N[k], (int)M, bf16,
                   p.slab, s));
      TTC_HIP(launch_core_perm(p.dWp, reinterpret_cast<float*>(dcores[k]), m->ranks[k], m->rows[k], m->cols[k],
                               m->ranks[k + 1], 1, s));
    }
    // dZ_k = dC_k Wp_k^T: B(k = n_fwd, n = (j, r)) = Wp_k[(j, r) * N + n_fwd]
    if (k > 0) {
      const IdxMap mp = step_map_inv(m, p, k - 1);
      TTC_TRY(gemm(true, dC, p.N[k], true, p.Wp[k], p.N[k], p.dC[(k - 1) & 1], 0, (int)M, (int)p.K[k],
                   (int)p.N[k], bf16, p.slab, s, &mp));
    } else if (dX) {
      TTC_TRY(gemm(true, dC, p.N[k], true, p.Wp[k], p.N[k], dX, p.K[k], (int)M, (int)p.K[k], (int)p.N[k], bf16,
                   p.slab, s));
    }
  }
  return TTC_OK;
}

// Validates the call and resolves the schedule (AUTO: fewer FLOPs).
ttc_status check_common(const ttc_ttm* m, int64_t batch, ttc_prec prec, ttc_sched sched, bool* bf16,
                        bool* cores, bool* saved = nullptr) {
  TTC_TRY(check_ttm(m));
  if (batch < 1 || batch > 2147483647LL) return fail(TTC_ERR_SHAPE, "batch outside [1, 2^31)");
  if (prec == TTC_PREC_BF16) *bf16 = true;
  else if (prec == TTC_PREC_AUTO || prec == TTC_PREC_F32) *bf16 = false;
  else return fail(TTC_ERR_UNSUPPORTED, "TT layer precision must be AUTO, F32 or BF16");
  if (sched != TTC_SCHED_AUTO && sched != TTC_SCHED_DENSE && sched != TTC_SCHED_CORES &&
      sched != TTC_SCHED_CORES_SAVED)
    return fail(TTC_ERR_UNSUPPORTED, "unknown schedule");
  if (saved) *saved = sched == TTC_SCHED_CORES_SAVED;
  CoresPlan cp;
  cores_shape(m, (long)batch, &cp);
  bool cores_ok = true;
  for (int k = 0; k < cp.d; ++k)
    if ((double)cp.P[k] * cp.Q[k] * std::max(cp.K[k], cp.N[k]) >= 9.2e18 / 8 ||
        (double)cp.P[k] * cp.Q[k] >= 2147483647.0)
      cores_ok = false;
  if ((sched == TTC_SCHED_CORES || sched == TTC_SCHED_CORES_SAVED) && !cores_ok)
    return fail(TTC_ERR_SHAPE, "core-by-core intermediates exceed 2^31 rows");
  *cores = sched == TTC_SCHED_CORES || sched == TTC_SCHED_CORES_SAVED ||
           (sched == TTC_SCHED_AUTO && cores_ok && cores_flops(cp) < dense_flops(m, (long)batch));
  return TTC_OK;
}

}  // namespace

namespace ttc {
ttc_status gemm_f32(bool a_kc, const float* A, long lda, bool b_kc, const float* B, long ldb, float* C, long ldc,
                    int M, int N, int K, float* slab, size_t slab_elems, hipStream_t s, const IdxMap* map) {
  return gemm(a_kc, A, lda, b_kc, B, ldb, C, ldc, M, N, K, false, slab, s, map, slab_elems);
}

ttc_status gemm_f32_batched(bool a_kc, const float* A, long lda, long sa, bool b_kc, const float* B, long ldb,
                            long sb, float* C, long ldc, long sc, int M, int N, int K, int batch, hipStream_t s,
                            const IdxMap* map) {
  if (batch < 1 || batch > 65535) return fail(TTC_ERR_SHAPE, "GEMM batch outside [1, 65535]");
  GemmArgs g;
  std::memset(&g, 0, sizeof(g));
  g.M = M;
  g.N = N;
  g.K = K;
  g.lda = lda;
  g.ldb = ldb;
  g.ldc = ldc;
  g.A = A;
  g.B = B;
  g.C = C;
  g.alpha = 1.f;
  g.splits = 1;
  g.batch = batch;
  g.sa = sa;
  g.sb = sb;
  g.sc = sc;
  if (map) {
    g.mapped = true;
    g.map = *map;
  }
  // vector loads need every batch member's operand 16-byte aligned too
  g.vec_a = (lda % 4 == 0) && (sa % 4 == 0) && aligned16(A);
  g.vec_b = (ldb % 4 == 0) && (sb % 4 == 0) && aligned16(B);
  g.tile = gemm_tile(M, N);
  TTC_HIP(launch_gemm(a_kc, b_kc, false, g, s));
  return TTC_OK;
}
}  // namespace ttc

extern "C" {

ttc_status ttm_apply_dense_query(const ttc_ttm* m, int64_t batch, ttc_prec prec, ttc_sched sched, int32_t backward,
                                 size_t* ws_bytes) {
  bool bf16 = false, cores = false, saved = false;
  TTC_TRY(check_common(m, batch, prec, sched, &bf16, &cores, &saved));
  if (!ws_bytes) return fail(TTC_ERR_NULL, "ws_bytes is NULL");
  Arena a(nullptr);
  if (cores) {
    CoresPlan p;
    plan_cores(m, (long)batch, backward != 0 || saved, a, &p);
  } else {
    LayerPlan p;
    plan_layer(m, backward != 0, bf16, (long)batch, a, &p);
  }
  *ws_bytes = a.off;
  return TTC_OK;
}

ttc_status ttm_apply_dense(const ttc_ttm* m, const void* d_x, int64_t batch, void* d_y, ttc_prec prec,
                           ttc_sched sched, void* d_ws, size_t ws_bytes, void* stream) {
  size_t need = 0;
  TTC_TRY(ttm_apply_dense_query(m, batch, prec, sched, 0, &need));
  if (!d_x || !d_y) return fail(TTC_ERR_NULL, "d_x or d_y is NULL");
  if (need > ws_bytes) return fail(TTC_ERR_WORKSPACE, "workspace smaller than ttm_apply_dense_query size");
  if (!d_ws) return fail(TTC_ERR_NULL, "d_ws is NULL");
  bool bf16 = false, cores = false, saved = false;
  TTC_TRY(check_common(m, batch, prec, sched, &bf16, &cores, &saved));
  hipStream_t s = (hipStream_t)stream;
  Arena a(d_ws);
  if (cores) {
    // saved: the backward's layout, every Z_k kept
    CoresPlan p;
    plan_cores(m, (long)batch, saved, a, &p);
    return cores_forward(m, p, reinterpret_cast<const float*>(d_x), reinterpret_cast<float*>(d_y), bf16, s);
  }
  LayerPlan p;
  plan_layer(m, false, bf16, (long)batch, a, &p);
  const float* X = reinterpret_cast<const float*>(d_x);
  if (bf16 && use_gemm16(batch, p.rows, p.cols) && aligned16(X)) {
    TTC_TRY(build_dense16(m, p, false, s));
    TTC_HIP(launch_cvt16(X, p.A16, (long)batch * p.cols, s));
    return gemm16(p.A16, p.cols, p.B16, p.cols, reinterpret_cast<float*>(d_y), p.rows, (int)batch, (int)p.rows,
                  (int)p.cols, s);
  }
  TTC_TRY(build_dense(m, p, s));
  // Y = X . W^T: A = X (batch x cols), B(k = j, n = i) = W[i * cols + j]
  return gemm(true, reinterpret_cast<const float*>(d_x), p.cols, true, p.Wd, p.cols, reinterpret_cast<float*>(d_y),
              p.rows, (int)batch, (int)p.rows, (int)p.cols, bf16, p.slab, s);
}

ttc_status ttm_apply_dense_bwd(const ttc_ttm* m, const void* d_x, const void* d_dy, int64_t batch, void* d_dx,
                               void* const* d_dcores, ttc_prec prec, ttc_sched sched, void* d_ws, size_t ws_bytes,
                               void* stream) {
  size_t need = 0;
  TTC_TRY(ttm_apply_dense_query(m, batch, prec, sched, 1, &need));
  if (!d_x || !d_dy) return fail(TTC_ERR_NULL, "d_x or d_dy is NULL");
  if (need > ws_bytes) return fail(TTC_ERR_WORKSPACE, "workspace smaller than ttm_apply_dense_query size");
  if (!d_ws) return fail(TTC_ERR_NULL, "d_ws is NULL");
  const int d = m->order;
  if (d_dcores)
    for (int k = 0; k < d; ++k)
      if (!d_dcores[k]) return fail(TTC_ERR_NULL, "NULL core-gradient buffer");
  bool bf16 = false, cores = false, saved = false;
  TTC_TRY(check_common(m, batch, prec, sched, &bf16, &cores, &saved));
  hipStream_t s = (hipStream_t)stream;
  Arena a(d_ws);
  if (cores) {
    CoresPlan p;
    plan_cores(m, (long)batch, true, a, &p);
    return cores_backward(m, p, reinterpret_cast<const float*>(d_x), reinterpret_cast<const float*>(d_dy),
                          reinterpret_cast<float*>(d_dx), d_dcores, bf16, saved, s);
  }
  LayerPlan p;
  plan_layer(m, true, bf16, (long)batch, a, &p);
  const float* X = reinterpret_cast<const float*>(d_x);
  const float* dY = reinterpret_cast<const float*>(d_dy);
  const bool al = aligned16(X) && aligned16(dY);
  const bool dx16 = d_dx && bf16 && al && use_gemm16(batch, p.cols, p.rows);
  const bool dw16 = d_dcores && bf16 && al && use_gemm16(p.rows, p.cols, batch);
  if (dx16)
    TTC_TRY(build_dense16(m, p, true, s));  // W^T in BF16
  else
    TTC_TRY(build_dense(m, p, s));
  if (dx16 && dw16) {
    // dY in both layouts from one read
    TTC_HIP(launch_cvt16_both(dY, p.A16, p.C16, batch, p.rows, s));
  } else if (dx16) {
    TTC_HIP(launch_cvt16(dY, p.A16, (long)batch * p.rows, s));
  }
  if (dx16) {
    // dX = dY . W: A = dY (batch x rows, k = i), B = W^T (cols x rows, k = i)
    TTC_TRY(gemm16(p.A16, p.rows, p.B16, p.rows, reinterpret_cast<float*>(d_dx), p.cols, (int)batch, (int)p.cols,
                   (int)p.rows, s));
  } else if (d_dx) {
    // dX = dY . W: A = dY (batch x rows), B(k = i, n = j) = W[i * cols + j]
    TTC_TRY(gemm(true, dY, p.rows, false, p.Wd, p.cols, reinterpret_cast<float*>(d_dx), p.cols, (int)batch,
                 (int)p.cols, (int)p.rows, bf16, p.slab, s));
  }
  if (!d_dcores) return TTC_OK;
  // dW = dY^T . X into the dense buffer: A(m = i, k = b) = dY[b * rows + i], B(k = b, n = j) = X[b * cols + j]
  if (dw16) {
    if (!dx16) TTC_HIP(launch_cvt16_t(dY, p.C16, batch, p.rows, s));
    TTC_HIP(launch_cvt16_t(X, p.D16, batch, p.cols, s));
    TTC_TRY(gemm16(p.C16, batch, p.D16, batch, p.Wd, p.cols, (int)p.rows, (int)p.cols, (int)batch, s));
  } else {
    TTC_TRY(gemm(false, dY, p.rows, false, X, p.cols, p.Wd, p.cols, (int)p.rows, (int)p.cols, (int)batch, bf16,
                 p.slab, s));
  }
  // dW -> pair-mode order (the right environment of the last core)
  TTC_TRY(permute_dense(m, 1, p.Wd, d == 1 ? reinterpret_cast<float*>(d_dcores[0]) : p.Dp, s));
  const float* Rt = p.Dp;  // Rt_{d-1}: |m_<d-1| x (M_{d-1} R_d)
  for (int k = d - 1; k >= 1; --k) {
    const long Mk = (long)m->rows[k] * m->cols[k];
    const int R = m->ranks[k], R1 = m->ranks[k + 1];
    const long n = Mk * R1;
    const int rowsL = (int)p.mprefix[k];
    // dG_k = L_k^T . Rt_k: A(m = r, k = a) = L_k[a * R + r], B(k = a, n) = Rt_k[a * n + n]
    TTC_TRY(gemm(false, p.L[k], R, false, Rt, n, reinterpret_cast<float*>(d_dcores[k]), n, R, (int)n, rowsL, false,
                 p.slab, s));
    // Rt_{k-1} = Rt_k . W^(k)^T: B(k = (m_k, r'), n = r) = W^(k)[r * n + k]
    float* nxt = (k == 1) ? reinterpret_cast<float*>(d_dcores[0]) : ((k % 2) ? p.RA : p.RB);
    TTC_TRY(gemm(true, Rt, n, true, reinterpret_cast<const float*>(m->cores[k]), n, nxt, R, rowsL, R, (int)n, false,
                 p.slab, s));
    Rt = nxt;
  }
  return TTC_OK;
}

ttc_status ttc_mse_loss_query(int64_t n, size_t* ws_bytes) {
  if (n < 1) return fail(TTC_ERR_SHAPE, "n < 1");
  if (!ws_bytes) return fail(TTC_ERR_NULL, "ws_bytes is NULL");
  *ws_bytes = (size_t)mse_blocks((long)n) * sizeof(double);
  return TTC_OK;
}

ttc_status ttc_mse_loss(const float* d_y, const float* d_t, int64_t n, double* d_loss, float* d_dy, void* d_ws,
                        size_t ws_bytes, void* stream) {
  size_t need = 0;
  TTC_TRY(ttc_mse_loss_query(n, &need));
  if (!d_y || !d_t || !d_loss) return fail(TTC_ERR_NULL, "d_y, d_t or d_loss is NULL");
  if (need > ws_bytes || !d_ws) return fail(TTC_ERR_WORKSPACE, "workspace smaller than ttc_mse_loss_query size");
  if (!aligned16(d_y) || !aligned16(d_t) || (d_dy && !aligned16(d_dy)))
    return fail(TTC_ERR_UNSUPPORTED, "buffers must be 16-byte aligned");
  TTC_HIP(launch_mse(d_y, d_t, (long)n, d_dy, reinterpret_cast<double*>(d_ws), d_loss, (hipStream_t)stream));
  return TTC_OK;
}

}  // extern "C"
