// Host side of TT-SVD (Algorithm 1): validation, workspace sizing and the
// N-1 splitting steps.  Each step runs the Jacobi SVD of the running
// unfolding on the GPU, reads the singular values back (the kept rank
// depends on them), picks the rank by the delta-truncation rule and splits
// the unfolding into core k and the next running matrix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "ttc_internal.h"

namespace ttc {
ttc_status fail(ttc_status s, const std::string& msg);
hipError_t launch_svd_transpose(ttc_dtype dt, const void* in, void* out, int m, int n, hipStream_t s);
hipError_t launch_svd_jacobi(ttc_dtype dt, void* A, void* J, double* sigma, int* info, int p, int L,
                             int max_sweeps, double tol, hipStream_t s);
hipError_t launch_svd_split(ttc_dtype dt, const void* A, const void* J, const double* sigma, const int* sel,
                            int tall, int m, int n, int p, int r, void* G, void* C, hipStream_t s);
hipError_t launch_svd_round(ttc_dtype dt, void* A, void* J, int p, int L, int rd, double tol, int* rotated,
                            hipStream_t s);
hipError_t launch_svd_ident(ttc_dtype dt, void* J, int p, hipStream_t s);
hipError_t launch_svd_norms(ttc_dtype dt, const void* A, double* sigma, int p, int L, hipStream_t s);
hipError_t launch_svd_rsplit(ttc_dtype dt, const void* A, const void* J, const double* sigma, const int* sel,
                             int tall, int m, int n, int p, int r, void* Q, void* B, hipStream_t s);
hipError_t launch_svd_small_gemm(ttc_dtype dt, const void* A, const void* B, void* C, long m, int K, long n,
                                 hipStream_t s);
}  // namespace ttc
using namespace ttc;

#define SVD_TRY(expr)            \
  do {                           \
    ttc_status _s = (expr);      \
    if (_s != TTC_OK) return _s; \
  } while (0)
#define SVD_HIP(expr)                                                                                    \
  do {                                                                                                   \
    hipError_t _e = (expr);                                                                              \
    if (_e != hipSuccess) return fail(TTC_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)

namespace {

// Largest number of vectors one Jacobi SVD rotates (min of the unfolding's
// sides); its p x p rotation matrix and sweeps grow with the square of it.
const long kMaxSvdVectors = 4096;
const int kMaxSweeps = 40;

struct SvdPlan {
  int N = 0;
  long numel = 1;
  std::vector<int> cap;  // rank capacity per bond (N + 1)
  long p_max = 1;
  size_t es = 8;
  size_t off_c0 = 0, off_c1 = 0, off_t = 0, off_j = 0, off_sigma = 0, off_sel = 0, off_info = 0, total = 0;
};

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Rotation threshold of the Jacobi SVD: a pair counts as orthogonal when
// |a_i . a_j| <= 32 u sqrt(L) ||a_i|| ||a_j|| for vectors of length L stored
// with unit roundoff u, a margin over the rounding level such normalised
// dot products reach (a tighter threshold keeps rotating pairs whose
// overlap is rounding noise).
double jacobi_tol(double unit, int L) { return 32.0 * unit * std::sqrt((double)std::max(L, 4)); }

// With TTC_SVD_TRACE set, one line per SVD on stderr: sweeps run and
// whether the last sweep rotated nothing.
void trace_sweeps(const char* who, int k, int p, int L, int sweeps, int converged) {
  static const bool on = std::getenv("TTC_SVD_TRACE") != nullptr;
  if (on) std::fprintf(stderr, "%s split %d: p %d L %d sweeps %d converged %d\n", who, k, p, L, sweeps, converged);
}

// Up to this many vectors one workgroup runs the whole Jacobi iteration
// (its rounds are short); above it each round is a launch with one
// workgroup per pair, so the p / 2 pairs of a round run on as many CUs.
const int kOneWorkgroupVectors = 32;

// Jacobi SVD of the p rows (length L) of A: rotations accumulated in J
// (p x p), row norms (the singular values) into sigma and then into sg on the
// host, in row order.  flag_d: two device ints of scratch.  Synchronises the
// stream at the end (and once per sweep on the many-workgroup path).
ttc_status jacobi_svd(ttc_dtype dt, void* A, void* J, double* sigma, int* flag_d, int p, int L, double tol,
                      hipStream_t s, std::vector<double>& sg, const char* who, int k) {
  int sweeps = 0, converged = 0;
  sg.assign(p, 0.0);
  if (p <= kOneWorkgroupVectors) {
    SVD_HIP(launch_svd_jacobi(dt, A, J, sigma, flag_d, p, L, kMaxSweeps, tol, s));
    int info[2] = {0, 0};
    SVD_HIP(hipMemcpyAsync(info, flag_d, sizeof(info), hipMemcpyDeviceToHost, s));
    SVD_HIP(hipMemcpyAsync(sg.data(), sigma, sizeof(double) * p, hipMemcpyDeviceToHost, s));
    SVD_HIP(hipStreamSynchronize(s));
    sweeps = info[0];
    converged = info[1];
  } else {
    SVD_HIP(launch_svd_ident(dt, J, p, s));
    const int rounds = p + (p & 1) - 1;
    while (sweeps < kMaxSweeps) {
      SVD_HIP(hipMemsetAsync(flag_d, 0, sizeof(int), s));
      for (int rd = 0; rd < rounds; ++rd) SVD_HIP(launch_svd_round(dt, A, J, p, L, rd, tol, flag_d, s));
      int flag = 0;
      SVD_HIP(hipMemcpyAsync(&flag, flag_d, sizeof(int), hipMemcpyDeviceToHost, s));
      SVD_HIP(hipStreamSynchronize(s));
      ++sweeps;
      if (!flag) {
        converged = 1;
        break;
      }
    }
    SVD_HIP(launch_svd_norms(dt, A, sigma, p, L, s));
    SVD_HIP(hipMemcpyAsync(sg.data(), sigma, sizeof(double) * p, hipMemcpyDeviceToHost, s));
    SVD_HIP(hipStreamSynchronize(s));
  }
  trace_sweeps(who, k, p, L, sweeps, converged);
  return TTC_OK;
}

ttc_status plan_svd(int32_t order, const int32_t* dims, ttc_dtype dtype, int32_t max_rank, SvdPlan* P) {
  if (order < 1 || order > TTC_MAX_ORDER) return fail(TTC_ERR_SHAPE, "tt_svd: order outside [1, 32]");
  if (!dims) return fail(TTC_ERR_NULL, "tt_svd: dims is NULL");
  if (dtype != TTC_F64 && dtype != TTC_F32) return fail(TTC_ERR_DTYPE, "tt_svd: FP64 or FP32 tensors");
  P->N = order;
  P->es = dtype == TTC_F64 ? 8 : 4;
  P->numel = 1;
  for (int k = 0; k < order; ++k) {
    if (dims[k] < 1) return fail(TTC_ERR_SHAPE, "tt_svd: mode size < 1");
    P->numel *= dims[k];
    if (P->numel > 2147483647L) return fail(TTC_ERR_UNSUPPORTED, "tt_svd: more than 2^31 - 1 entries");
  }
  P->cap.assign(order + 1, 1);
  long rest = P->numel;
  P->p_max = 1;
  for (int k = 0; k + 1 < order; ++k) {
    const long m = (long)P->cap[k] * dims[k];
    rest /= dims[k];
    const long p = std::min(m, rest);
    P->p_max = std::max(P->p_max, p);
    long c = p;
    if (max_rank > 0) c = std::min<long>(c, max_rank);
    P->cap[k + 1] = (int)c;
  }
  if (P->p_max > kMaxSvdVectors)
    return fail(TTC_ERR_UNSUPPORTED, "tt_svd: an unfolding has more than " + std::to_string(kMaxSvdVectors) +
                                         " rows and columns (min side " + std::to_string(P->p_max) + ")");
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  P->off_c0 = take(P->numel * P->es);
  P->off_c1 = take(P->numel * P->es);
  P->off_t = take(P->numel * P->es);
  P->off_j = take((size_t)P->p_max * P->p_max * P->es);
  P->off_sigma = take((size_t)P->p_max * sizeof(double));
  P->off_sel = take((size_t)P->p_max * sizeof(int));
  P->off_info = take(2 * sizeof(int));
  P->total = off;
  return TTC_OK;
}

}  // namespace

extern "C" {

ttc_status tt_svd_query(int32_t order, const int32_t* dims, ttc_dtype dtype, int32_t max_rank, int32_t* rank_cap,
                        size_t* ws_bytes) {
  SvdPlan P;
  SVD_TRY(plan_svd(order, dims, dtype, max_rank, &P));
  if (rank_cap)
    for (int k = 0; k <= order; ++k) rank_cap[k] = P.cap[k];
  if (ws_bytes) *ws_bytes = P.total;
  return TTC_OK;
}

ttc_status tt_svd(const void* d_x, int32_t order, const int32_t* dims, ttc_dtype dtype, double eps,
                  int32_t max_rank, int32_t* ranks, void* const* d_cores, void* d_ws, size_t ws_bytes,
                  void* stream) {
  SvdPlan P;
  SVD_TRY(plan_svd(order, dims, dtype, max_rank, &P));
  if (!d_x) return fail(TTC_ERR_NULL, "tt_svd: d_x is NULL");
  if (!ranks || !d_cores) return fail(TTC_ERR_NULL, "tt_svd: ranks or d_cores is NULL");
  for (int k = 0; k < order; ++k)
    if (!d_cores[k]) return fail(TTC_ERR_NULL, "tt_svd: NULL core buffer");
  if (!(eps >= 0.0) || !std::isfinite(eps)) return fail(TTC_ERR_SHAPE, "tt_svd: eps must be finite and >= 0");
  if (P.total > ws_bytes) return fail(TTC_ERR_WORKSPACE, "workspace smaller than tt_svd_query size");
  if (!d_ws) return fail(TTC_ERR_NULL, "tt_svd: d_ws is NULL");
  hipStream_t s = (hipStream_t)stream;
  char* ws = static_cast<char*>(d_ws);
  void* cur = ws + P.off_c0;
  void* nxt = ws + P.off_c1;
  void* tbuf = ws + P.off_t;
  void* J = ws + P.off_j;
  double* sigma = reinterpret_cast<double*>(ws + P.off_sigma);
  int* sel_d = reinterpret_cast<int*>(ws + P.off_sel);
  int* info_d = reinterpret_cast<int*>(ws + P.off_info);
  const int N = order;
  std::vector<int> rk(N + 1, 1);
  if (N == 1) {
    SVD_HIP(hipMemcpyAsync(d_cores[0], d_x, P.numel * P.es, hipMemcpyDeviceToDevice, s));
    ranks[0] = ranks[1] = 1;
    return TTC_OK;
  }
  SVD_HIP(hipMemcpyAsync(cur, d_x, P.numel * P.es, hipMemcpyDeviceToDevice, s));
  // Jacobi stopping threshold: the rounding level of a dot product of two
  // rows of length L in the storage precision
  const double unit = dtype == TTC_F64 ? 1.1102230246251565e-16 : 5.960464477539063e-08;
  double delta = 0.0;
  long cur_elems = P.numel;
  std::vector<double> sg;
  std::vector<int> order_idx;
  for (int k = 0; k + 1 < N; ++k) {
    const long m = (long)rk[k] * dims[k];
    const long n = cur_elems / m;
    const bool tall = m > n;
    const int p = (int)std::min(m, n), L = (int)std::max(m, n);
    void* A = cur;
    if (tall) {
      SVD_HIP(launch_svd_transpose(dtype, cur, tbuf, (int)m, (int)n, s));
      A = tbuf;
    }
    SVD_TRY(jacobi_svd(dtype, A, J, sigma, info_d, p, L, jacobi_tol(unit, L), s, sg, "tt_svd", k));
    if (k == 0) {
      // ||X||_F from the first unfolding's singular values
      double nx2 = 0;
      for (double v : sg) nx2 += v * v;
      delta = eps / std::sqrt((double)(N - 1)) * std::sqrt(nx2);
    }
    order_idx.resize(p);
    std::iota(order_idx.begin(), order_idx.end(), 0);
    std::stable_sort(order_idx.begin(), order_idx.end(), [&](int a, int b) { return sg[a] > sg[b]; });
    // smallest r >= 1 whose discarded singular values have norm <= delta
    std::vector<double> tail(p + 1, 0.0);
    for (int c = p - 1; c >= 0; --c) tail[c] = tail[c + 1] + sg[order_idx[c]] * sg[order_idx[c]];
    int r = p;
    for (int c = 1; c <= p; ++c)
      if (std::sqrt(tail[c]) <= delta) {
        r = c;
        break;
      }
    r = std::min(r, P.cap[k + 1]);
    SVD_HIP(hipMemcpy(sel_d, order_idx.data(), sizeof(int) * r, hipMemcpyHostToDevice));
    SVD_HIP(launch_svd_split(dtype, A, J, sigma, sel_d, tall ? 1 : 0, (int)m, (int)n, p, r, d_cores[k], nxt, s));
    rk[k + 1] = r;
    std::swap(cur, nxt);
    cur_elems = (long)r * n;
  }
  SVD_HIP(hipMemcpyAsync(d_cores[N - 1], cur, cur_elems * P.es, hipMemcpyDeviceToDevice, s));
  for (int k = 0; k <= N; ++k) ranks[k] = rk[k];
  return TTC_OK;
}


}  // extern "C"

// ---------------------------------------------------------------------------
// TT-rounding: the same delta-truncation applied to a TT given by its cores.
// Right to left, each core's unfolding (left bond x the rest) is split by
// the Jacobi SVD into orthonormal rows Q (the new core) and B = U S, which
// is multiplied into the core on its left; then left to right, exactly as in
// tt_svd, each core's unfolding is split, core k keeps the left singular
// vectors and S V^T is multiplied into core k + 1.  After the first pass
// every core right of the current one is right-orthonormal, so the singular
// values at each bond are those of the tensor's unfolding there, and the
// result is what tt_svd gives on the full tensor (up to signs).
// ---------------------------------------------------------------------------
namespace {

struct RoundPlan {
  int N = 0;
  size_t es = 8;
  long max_core = 1;
  long p_max = 1;
  std::vector<int> cap;
  size_t off_cores = 0, core_bytes = 0, off_t = 0, off_b = 0, off_j = 0, off_sigma = 0, off_sel = 0, off_info = 0;
  size_t total = 0;
};

ttc_status plan_round(const ttc_tt* x, int32_t max_rank, RoundPlan* P) {
  if (!x) return fail(TTC_ERR_NULL, "tt_round: x is NULL");
  if (x->order < 1 || x->order > TTC_MAX_ORDER) return fail(TTC_ERR_SHAPE, "tt_round: order outside [1, 32]");
  if (!x->modes || !x->ranks || !x->cores) return fail(TTC_ERR_NULL, "tt_round: NULL descriptor array");
  if (x->dtype != TTC_F64 && x->dtype != TTC_F32) return fail(TTC_ERR_DTYPE, "tt_round: FP64 or FP32 cores");
  const int N = x->order;
  if (x->ranks[0] != 1 || x->ranks[N] != 1) return fail(TTC_ERR_RANK, "tt_round: boundary ranks must be 1");
  P->N = N;
  P->es = x->dtype == TTC_F64 ? 8 : 4;
  P->max_core = 1;
  P->p_max = 1;
  for (int k = 0; k < N; ++k) {
    if (x->modes[k] < 1 || x->ranks[k] < 1) return fail(TTC_ERR_SHAPE, "tt_round: bad shape");
    if (!x->cores[k]) return fail(TTC_ERR_NULL, "tt_round: NULL core pointer");
    const long r0 = x->ranks[k], n = x->modes[k], r1 = x->ranks[k + 1];
    if ((double)r0 * n * r1 >= 2147483647.0) return fail(TTC_ERR_SHAPE, "tt_round: core too large");
    P->max_core = std::max(P->max_core, r0 * n * r1);
    P->p_max = std::max(P->p_max, std::min(r0, n * r1));
    P->p_max = std::max(P->p_max, std::min(r0 * n, r1));
  }
  if (P->p_max > kMaxSvdVectors)
    return fail(TTC_ERR_UNSUPPORTED, "tt_round: a core unfolding has more than " + std::to_string(kMaxSvdVectors) +
                                         " rows and columns");
  // bond capacities: the input rank, and the rank either side's modes allow
  P->cap.assign(N + 1, 1);
  double left = 1;
  for (int k = 1; k < N; ++k) {
    left *= x->modes[k - 1];
    double right = 1;
    for (int j = k; j < N; ++j) right *= x->modes[j];
    double c = std::min<double>({(double)x->ranks[k], left, right});
    if (max_rank > 0) c = std::min<double>(c, max_rank);
    P->cap[k] = (int)c;
  }
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  P->core_bytes = align256((size_t)P->max_core * P->es);
  P->off_cores = take(P->core_bytes * (N + 1));  // N working cores and one spare
  P->off_t = take((size_t)P->max_core * P->es);
  P->off_b = take((size_t)P->max_core * P->es);
  P->off_j = take((size_t)P->p_max * P->p_max * P->es);
  P->off_sigma = take((size_t)P->p_max * sizeof(double));
  P->off_sel = take((size_t)P->p_max * sizeof(int));
  P->off_info = take(2 * sizeof(int));
  P->total = off;
  return TTC_OK;
}

// Jacobi SVD of the m x n row-major matrix at M (a transposed copy in tbuf
// when m > n); singular values returned in decreasing order (sg, order).
ttc_status svd_of(ttc_dtype dt, void* M, long m, long n, char* ws, const RoundPlan& P, hipStream_t s, void** A,
                  bool* tall, std::vector<double>& sg, std::vector<int>& order) {
  const double unit = dt == TTC_F64 ? 1.1102230246251565e-16 : 5.960464477539063e-08;
  *tall = m > n;
  const int p = (int)std::min(m, n), L = (int)std::max(m, n);
  *A = M;
  if (*tall) {
    SVD_HIP(launch_svd_transpose(dt, M, ws + P.off_t, (int)m, (int)n, s));
    *A = ws + P.off_t;
  }
  SVD_TRY(jacobi_svd(dt, *A, ws + P.off_j, reinterpret_cast<double*>(ws + P.off_sigma),
                     reinterpret_cast<int*>(ws + P.off_info), p, L, jacobi_tol(unit, L), s, sg, "tt_round", 0));
  order.resize(p);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return sg[a] > sg[b]; });
  return TTC_OK;
}

}  // namespace

extern "C" {

ttc_status tt_round_query(const ttc_tt* x, int32_t max_rank, int32_t* rank_cap, size_t* ws_bytes) {
  RoundPlan P;
  SVD_TRY(plan_round(x, max_rank, &P));
  if (rank_cap)
    for (int k = 0; k <= x->order; ++k) rank_cap[k] = P.cap[k];
  if (ws_bytes) *ws_bytes = P.total;
  return TTC_OK;
}

ttc_status tt_round(const ttc_tt* x, double eps, int32_t max_rank, int32_t* ranks, void* const* d_cores,
                    void* d_ws, size_t ws_bytes, void* stream) {
  RoundPlan P;
  SVD_TRY(plan_round(x, max_rank, &P));
  const int N = x->order;
  if (!ranks || !d_cores) return fail(TTC_ERR_NULL, "tt_round: ranks or d_cores is NULL");
  for (int k = 0; k < N; ++k)
    if (!d_cores[k]) return fail(TTC_ERR_NULL, "tt_round: NULL output core");
  if (!(eps >= 0.0) || !std::isfinite(eps)) return fail(TTC_ERR_SHAPE, "tt_round: eps must be finite and >= 0");
  if (P.total > ws_bytes) return fail(TTC_ERR_WORKSPACE, "workspace smaller than tt_round_query size");
  if (!d_ws) return fail(TTC_ERR_NULL, "tt_round: d_ws is NULL");
  hipStream_t s = (hipStream_t)stream;
  const ttc_dtype dt = x->dtype;
  char* ws = static_cast<char*>(d_ws);
  std::vector<void*> W(N + 1);
  for (int k = 0; k <= N; ++k) W[k] = ws + P.off_cores + (size_t)k * P.core_bytes;
  void* spare = W[N];
  std::vector<int> r(N + 1);
  for (int k = 0; k <= N; ++k) r[k] = x->ranks[k];
  for (int k = 0; k < N; ++k)
    SVD_HIP(hipMemcpyAsync(W[k], x->cores[k], (size_t)r[k] * x->modes[k] * r[k + 1] * P.es,
                           hipMemcpyDeviceToDevice, s));
  if (N == 1) {
    SVD_HIP(hipMemcpyAsync(d_cores[0], W[0], (size_t)x->modes[0] * P.es, hipMemcpyDeviceToDevice, s));
    ranks[0] = ranks[1] = 1;
    return TTC_OK;
  }
  int* sel_d = reinterpret_cast<int*>(ws + P.off_sel);
  const double* sigma_d = reinterpret_cast<const double*>(ws + P.off_sigma);
  void* B = ws + P.off_b;
  std::vector<double> sg;
  std::vector<int> order;
  // right to left: core k = B Q, Q orthonormal rows; B into core k - 1
  for (int k = N - 1; k >= 1; --k) {
    const long m = r[k], n = (long)x->modes[k] * r[k + 1];
    void* A = nullptr;
    bool tall = false;
    SVD_TRY(svd_of(dt, W[k], m, n, ws, P, s, &A, &tall, sg, order));
    int rk = 0;
    for (double v : sg) rk += v > 0 ? 1 : 0;
    rk = std::max(rk, 1);
    SVD_HIP(hipMemcpy(sel_d, order.data(), sizeof(int) * rk, hipMemcpyHostToDevice));
    const int p = (int)std::min(m, n);
    SVD_HIP(launch_svd_rsplit(dt, A, ws + P.off_j, sigma_d, sel_d, tall ? 1 : 0, (int)m, (int)n, p, rk, spare, B, s));
    std::swap(W[k], spare);
    // core k - 1 (R_{k-1} I_{k-1} x R_k) times B (R_k x rk)
    const long lm = (long)r[k - 1] * x->modes[k - 1];
    SVD_HIP(launch_svd_small_gemm(dt, W[k - 1], B, spare, lm, (int)m, rk, s));
    std::swap(W[k - 1], spare);
    r[k] = rk;
  }
  // left to right: the delta-truncated splits of tt_svd
  double delta = 0.0;
  for (int k = 0; k + 1 < N; ++k) {
    const long m = (long)r[k] * x->modes[k], n = r[k + 1];
    void* A = nullptr;
    bool tall = false;
    SVD_TRY(svd_of(dt, W[k], m, n, ws, P, s, &A, &tall, sg, order));
    const int p = (int)std::min(m, n);
    if (k == 0) {
      double nx2 = 0;
      for (double v : sg) nx2 += v * v;
      delta = eps / std::sqrt((double)(N - 1)) * std::sqrt(nx2);
    }
    std::vector<double> tail(p + 1, 0.0);
    for (int c = p - 1; c >= 0; --c) tail[c] = tail[c + 1] + sg[order[c]] * sg[order[c]];
    int rk = p;
    for (int c = 1; c <= p; ++c)
      if (std::sqrt(tail[c]) <= delta) {
        rk = c;
        break;
      }
    rk = std::min(rk, P.cap[k + 1]);
    SVD_HIP(hipMemcpy(sel_d, order.data(), sizeof(int) * rk, hipMemcpyHostToDevice));
    // core k = U_rk (into the caller's buffer), S V^T (rk x R_{k+1}) into B
    SVD_HIP(launch_svd_split(dt, A, ws + P.off_j, sigma_d, sel_d, tall ? 1 : 0, (int)m, (int)n, p, rk, d_cores[k], B,
                             s));
    const long rn = (long)x->modes[k + 1] * r[k + 2];
    SVD_HIP(launch_svd_small_gemm(dt, B, W[k + 1], spare, rk, (int)n, rn, s));
    std::swap(W[k + 1], spare);
    r[k + 1] = rk;
  }
  SVD_HIP(hipMemcpyAsync(d_cores[N - 1], W[N - 1], (size_t)r[N - 1] * x->modes[N - 1] * P.es,
                         hipMemcpyDeviceToDevice, s));
  for (int k = 0; k <= N; ++k) ranks[k] = r[k];
  return TTC_OK;
}

}  // extern "C"
