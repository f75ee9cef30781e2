// Host-side ABI checks for a build with AddressSanitizer and
// UndefinedBehaviorSanitizer on the host code: every query and validation
// path of the library, with valid and invalid descriptors.  No call here
// reaches the device (queries and rejected calls return before any launch),
// so the program runs without a GPU.  Exits non-zero on a wrong status; the
// sanitizers abort on any memory or undefined-behaviour error.
#include <cstdint>
#include <cstdio>
#include <vector>

#include "../../include/ttc.h"

namespace {

int failures = 0;

void expect(const char* what, ttc_status got, ttc_status want) {
  if (got != want) {
    std::printf("FAIL %s: status %d, expected %d (%s)\n", what, (int)got, (int)want, ttc_last_error());
    ++failures;
  }
}

// A TT descriptor with fake core pointers (never dereferenced).
struct Tt {
  std::vector<int32_t> modes, ranks;
  std::vector<void*> cores;
  ttc_tt d;
  Tt(std::vector<int32_t> m, std::vector<int32_t> r, ttc_dtype dt = TTC_F32) : modes(m), ranks(r) {
    for (size_t k = 0; k < modes.size(); ++k) cores.push_back(reinterpret_cast<void*>(0x7f0000001000ull + 4096 * k));
    d.order = (int32_t)modes.size();
    d.modes = modes.data();
    d.ranks = ranks.data();
    d.dtype = dt;
    d.cores = cores.data();
  }
};

// Deterministic shapes of the uneven batch's kind (a 64-bit LCG).
uint64_t lcg = 88172645463325252ull;
int draw(int lo, int hi) {
  lcg = lcg * 6364136223846793005ull + 1442695040888963407ull;
  return lo + (int)((lcg >> 33) % (uint64_t)(hi - lo + 1));
}

}  // namespace

int main() {
  size_t ws = 0;
  // inner products: valid, and every kind of bad descriptor
  Tt x({4, 5, 6, 3}, {1, 3, 4, 2, 1}), y({4, 5, 6, 3}, {1, 2, 5, 3, 1});
  expect("inner query", tt_contract_inner_query(&x.d, &y.d, TTC_PREC_AUTO, &ws), TTC_OK);
  Tt bad_rank({4, 5}, {2, 3, 1});
  expect("boundary rank", tt_contract_inner_query(&bad_rank.d, &bad_rank.d, TTC_PREC_AUTO, &ws), TTC_ERR_RANK);
  Tt other({4, 5, 7, 3}, {1, 2, 5, 3, 1});
  expect("mode mismatch", tt_contract_inner_query(&x.d, &other.d, TTC_PREC_AUTO, &ws), TTC_ERR_SHAPE);
  expect("null ws", tt_contract_inner_query(&x.d, &y.d, TTC_PREC_AUTO, nullptr), TTC_ERR_NULL);
  if (ws > 0)
    expect("inner workspace", tt_contract_inner(&x.d, &y.d, TTC_PREC_AUTO, reinterpret_cast<double*>(0x1000),
                                                nullptr, 0, nullptr),
           TTC_ERR_WORKSPACE);
  // shared-position contractions in every form
  const int32_t pre[2] = {0, 1}, suf[2] = {2, 3}, mid[1] = {1}, rep[2] = {1, 1};
  int32_t order = 0, om[16], orr[17];
  int64_t elems = 0;
  for (int f = 0; f < 3; ++f) {
    expect("modes prefix",
           tt_contract_modes_query(&x.d, &y.d, pre, 2, (ttc_form)f, TTC_PREC_AUTO, &order, om, orr, &elems, &ws),
           TTC_OK);
    expect("modes suffix",
           tt_contract_modes_query(&x.d, &y.d, suf, 2, (ttc_form)f, TTC_PREC_AUTO, &order, om, orr, &elems, &ws),
           TTC_OK);
  }
  expect("modes middle",
         tt_contract_modes_query(&x.d, &y.d, mid, 1, TTC_JUNCTION, TTC_PREC_AUTO, &order, om, orr, &elems, &ws),
         TTC_ERR_UNSUPPORTED);
  expect("modes repeat",
         tt_contract_modes_query(&x.d, &y.d, rep, 2, TTC_JUNCTION, TTC_PREC_AUTO, &order, om, orr, &elems, &ws),
         TTC_ERR_MODE);
  expect("modes bf16 prec on fp32",
         tt_contract_modes_query(&x.d, &y.d, pre, 2, TTC_JUNCTION, TTC_PREC_BF16, &order, om, orr, &elems, &ws),
         TTC_ERR_UNSUPPORTED);
  // contractions at any positions, every form
  Tt a({3, 4, 5, 2}, {1, 2, 3, 2, 1}), b({3, 5, 4}, {1, 2, 3, 1});
  const int32_t xm[1] = {2}, ym[1] = {1}, xm2[2] = {0, 2}, ym2[2] = {0, 1};
  for (int f = 0; f < 3; ++f)
    expect("pairs", tt_contract_pairs_query(&a.d, &b.d, xm, ym, 1, (ttc_form)f, &order, om, orr, &elems, &ws),
           TTC_OK);
  expect("pairs gap", tt_contract_pairs_query(&a.d, &b.d, xm2, ym2, 2, TTC_JUNCTION, &order, om, orr, &elems, &ws),
         TTC_ERR_UNSUPPORTED);
  // mode-n, MPO, layer, loss, gradient queries
  const int32_t rows[3] = {4, 3, 2}, cols[3] = {3, 4, 2}, wr[4] = {1, 3, 2, 1};
  void* wc[3] = {reinterpret_cast<void*>(0x7f0000100000ull), reinterpret_cast<void*>(0x7f0000200000ull),
                 reinterpret_cast<void*>(0x7f0000300000ull)};
  ttc_ttm w{3, rows, cols, wr, TTC_F32, wc};
  Tt v({3, 4, 2}, {1, 2, 2, 1});
  int32_t out_ranks[4];
  expect("mpo query", ttm_apply_query(&w, &v.d, out_ranks, &elems), TTC_OK);
  expect("dense query", ttm_apply_dense_query(&w, 37, TTC_PREC_AUTO, TTC_SCHED_CORES, 1, &ws), TTC_OK);
  expect("dense query dense", ttm_apply_dense_query(&w, 37, TTC_PREC_BF16, TTC_SCHED_DENSE, 1, &ws), TTC_OK);
  expect("dense query saved", ttm_apply_dense_query(&w, 37, TTC_PREC_AUTO, TTC_SCHED_CORES_SAVED, 0, &ws), TTC_OK);
  expect("mse query", ttc_mse_loss_query(1001, &ws), TTC_OK);
  for (int c = 0; c <= 4; ++c) expect("grad query", tt_contract_inner_bwd_query(&x.d, &y.d, c, &ws), TTC_OK);
  // TT-SVD and rounding queries
  const int32_t dims[5] = {20, 20, 20, 5, 4};
  int32_t cap[6];
  expect("svd query", tt_svd_query(5, dims, TTC_F64, 0, cap, &ws), TTC_OK);
  expect("svd dtype", tt_svd_query(5, dims, TTC_BF16, 0, cap, &ws), TTC_ERR_DTYPE);
  Tt r({4, 5, 6, 3}, {1, 4, 8, 3, 1}, TTC_F64);
  expect("round query", tt_round_query(&r.d, 0, cap, &ws), TTC_OK);
  // the batch planner's host bookkeeping on 500 uneven pairs
  std::vector<Tt> xs, ys;
  xs.reserve(500);
  ys.reserve(500);
  for (int p = 0; p < 500; ++p) {
    const int N = draw(3, 12);
    std::vector<int32_t> m(N), rx(N + 1, 1), ry(N + 1, 1);
    for (int k = 0; k < N; ++k) m[k] = 4 << draw(0, 4);
    for (int k = 1; k < N; ++k) {
      rx[k] = draw(8, 128);
      ry[k] = draw(8, 128);
    }
    xs.emplace_back(m, rx);
    ys.emplace_back(m, ry);
  }
  std::vector<ttc_pair> pairs;
  for (int p = 0; p < 500; ++p) pairs.push_back(ttc_pair{xs[p].d, ys[p].d});
  std::vector<int64_t> joff(501);
  std::vector<double> cost(500);
  std::vector<int32_t> claim(500);
  double fl = 0, by = 0;
  expect("plan query", tt_batch_plan_query(pairs.data(), 500, 3, joff.data(), &fl, &by, cost.data(), claim.data()),
         TTC_OK);
  for (int i = 1; i < 500; ++i)
    if (cost[claim[i - 1]] < cost[claim[i]]) {
      std::printf("FAIL claim order at %d\n", i);
      ++failures;
      break;
    }
  expect("plan query no ops", tt_batch_plan_query(pairs.data(), 500, 0, nullptr, nullptr, nullptr, nullptr, nullptr),
         TTC_ERR_UNSUPPORTED);
  expect("plan null", tt_batch_plan_query(nullptr, 5, 3, nullptr, nullptr, nullptr, nullptr, nullptr), TTC_ERR_NULL);
  std::printf("%s: %d failure(s)\n", failures ? "FAIL" : "ok", failures);
  return failures ? 1 : 0;
}
