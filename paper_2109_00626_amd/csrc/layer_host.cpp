// Host side of the TT layer: TT-matrix x dense batch (forward, backward)
// and the MSE loss.  See layer.hip for the schedule.
#include <hip/hip_runtime.h>

#include <algorithm>
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
};

void plan_layer(const ttc_ttm* m, bool backward, Arena& a, LayerPlan* p) {
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
}

bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

// One GEMM with split-K chosen to give the GPU enough workgroups.
ttc_status gemm(bool a_kc, const float* A, long lda, bool b_kc, const float* B, long ldb, float* C, long ldc, int M,
                int N, int K, bool bf16, float* slab, hipStream_t s) {
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
  g.vec_a = (lda % 4 == 0) && aligned16(A);
  g.vec_b = (ldb % 4 == 0) && aligned16(B);
  const long tiles = (long)((M + 127) / 128) * ((N + 127) / 128);
  const int bk = gemm_bk(bf16);
  int splits = 1;
  if (tiles < 512) {
    long want = (1024 + tiles - 1) / tiles;
    long by_k = K / (4L * bk);
    long by_slab = (long)(kSlabElems / ((size_t)M * N));
    splits = (int)std::max(1L, std::min(want, std::min(by_k, by_slab)));
  }
  g.splits = splits;
  g.slab = slab;
  TTC_HIP(launch_gemm(a_kc, b_kc, bf16, g, s));
  return TTC_OK;
}

// Dense matrix W[i, j] from the cores: chain L_{k+1} = L_k . W^(k), then the
// pair-mode -> matrix permutation.  Keeps every L_k in the plan.
ttc_status build_dense(const ttc_ttm* m, LayerPlan& p, hipStream_t s) {
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
  PermArgs pa;
  std::memset(&pa, 0, sizeof(pa));
  pa.dir = 0;
  pa.d = d;
  for (int k = 0; k < d; ++k) {
    pa.I[k] = m->rows[k];
    pa.J[k] = m->cols[k];
  }
  pa.pstride[d - 1] = 1;
  for (int k = d - 2; k >= 0; --k) pa.pstride[k] = pa.pstride[k + 1] * m->rows[k + 1] * m->cols[k + 1];
  pa.cols = p.cols;
  pa.total = p.rows * p.cols;
  pa.src = d == 1 ? reinterpret_cast<const float*>(m->cores[0]) : p.Dp;
  pa.dst = p.Wd;
  TTC_HIP(launch_permute(pa, s));
  return TTC_OK;
}

ttc_status check_common(const ttc_ttm* m, int64_t batch, ttc_prec prec, ttc_sched sched, bool* bf16) {
  TTC_TRY(check_ttm(m));
  if (batch < 1 || batch > 2147483647LL) return fail(TTC_ERR_SHAPE, "batch outside [1, 2^31)");
  if (prec == TTC_PREC_BF16) *bf16 = true;
  else if (prec == TTC_PREC_AUTO || prec == TTC_PREC_F32) *bf16 = false;
  else return fail(TTC_ERR_UNSUPPORTED, "TT layer precision must be AUTO, F32 or BF16");
  if (sched == TTC_SCHED_CORES) return fail(TTC_ERR_UNSUPPORTED, "core-by-core schedule not available");
  if (sched != TTC_SCHED_AUTO && sched != TTC_SCHED_DENSE) return fail(TTC_ERR_UNSUPPORTED, "unknown schedule");
  return TTC_OK;
}

}  // namespace

extern "C" {

ttc_status ttm_apply_dense_query(const ttc_ttm* m, int64_t batch, ttc_prec prec, ttc_sched sched, int32_t backward,
                                 size_t* ws_bytes) {
  bool bf16 = false;
  TTC_TRY(check_common(m, batch, prec, sched, &bf16));
  if (!ws_bytes) return fail(TTC_ERR_NULL, "ws_bytes is NULL");
  Arena a(nullptr);
  LayerPlan p;
  plan_layer(m, backward != 0, a, &p);
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
  bool bf16 = prec == TTC_PREC_BF16;
  hipStream_t s = (hipStream_t)stream;
  Arena a(d_ws);
  LayerPlan p;
  plan_layer(m, false, a, &p);
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
  bool bf16 = prec == TTC_PREC_BF16;
  hipStream_t s = (hipStream_t)stream;
  Arena a(d_ws);
  LayerPlan p;
  plan_layer(m, true, a, &p);
  TTC_TRY(build_dense(m, p, s));
  const float* X = reinterpret_cast<const float*>(d_x);
  const float* dY = reinterpret_cast<const float*>(d_dy);
  if (d_dx) {
    // dX = dY . W: A = dY (batch x rows), B(k = i, n = j) = W[i * cols + j]
    TTC_TRY(gemm(true, dY, p.rows, false, p.Wd, p.cols, reinterpret_cast<float*>(d_dx), p.cols, (int)batch,
                 (int)p.cols, (int)p.rows, bf16, p.slab, s));
  }
  if (!d_dcores) return TTC_OK;
  // dW = dY^T . X into the dense buffer: A(m = i, k = b) = dY[b * rows + i], B(k = b, n = j) = X[b * cols + j]
  TTC_TRY(gemm(false, dY, p.rows, false, X, p.cols, p.Wd, p.cols, (int)p.rows, (int)p.cols, (int)batch, bf16,
               p.slab, s));
  // dW -> pair-mode order (the right environment of the last core)
  PermArgs pa;
  std::memset(&pa, 0, sizeof(pa));
  pa.dir = 1;
  pa.d = d;
  for (int k = 0; k < d; ++k) {
    pa.I[k] = m->rows[k];
    pa.J[k] = m->cols[k];
  }
  pa.pstride[d - 1] = 1;
  for (int k = d - 2; k >= 0; --k) pa.pstride[k] = pa.pstride[k + 1] * m->rows[k + 1] * m->cols[k + 1];
  pa.cols = p.cols;
  pa.total = p.rows * p.cols;
  pa.src = p.Wd;
  pa.dst = d == 1 ? reinterpret_cast<float*>(d_dcores[0]) : p.Dp;
  TTC_HIP(launch_permute(pa, s));
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
