// Host side of the batched sweep: validation, cost model, longest-first
// assignment of pairs to persistent workgroups, descriptor upload, launch
// shape selection by timing (the autotuner), HIP-graph capture and replay,
// and the per-pair launch loop used as the unbatched reference.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <functional>
#include <map>
#include <mutex>
#include <queue>
#include <sstream>
#include <string>
#include <vector>

#include "ttc_batch.h"

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

struct PairHost {
  int order;
  std::vector<int> modes, rx, ry;
  std::vector<void*> xc, yc;
};

// One launch shape: workgroup size and workgroups per compute unit.
struct LaunchCfg {
  int mode = 2;
  int threads = 256;
  int per_cu = 1;
};

struct ttc_plan {
  int n = 0;
  uint32_t ops = 0;
  ttc_dtype dt = TTC_F32;
  ttc_prec prec = TTC_PREC_AUTO;  // BF16: BF16-MFMA steps only; F32: FP32-MFMA steps only
  int device = 0;
  int cus = 256;
  std::vector<PairHost> pairs;
  std::vector<int64_t> joff;
  std::vector<double> cost;
  double flops = 0, bytes = 0;
  long max_rp = 1, max_t = 1;
  // device memory (one allocation for the tables, one for the level buffers)
  void* dmem = nullptr;
  void* dmem_levels = nullptr;
  PairDev* d_pairs = nullptr;
  int* d_ipool = nullptr;
  void** d_ppool = nullptr;
  int* d_begin = nullptr;   // per configuration, rebuilt on selection
  int* d_order = nullptr;
  int* d_ident = nullptr;   // 0..n-1 (per-pair launches)
  int* d_01 = nullptr;      // {0, 1}
  int* d_claim = nullptr;   // LDS-resident kernels: work counter and exit count (zero between launches)
  float* d_iface = nullptr;
  float* d_tbuf = nullptr;
  int max_grid = 0;
  // selected launch
  LaunchCfg cfg;
  int grid = 0;
  int lds_elems = 0;
  // level-by-level execution
  int mode = 0;                // 0: persistent kernel, 1: one launch per level, 2: LDS-resident persistent
                               // kernel, 3: the same with one interface buffer updated in place
  int buf_elems = 0;           // LDS-resident kernel: floats per interface buffer
  int stage16 = 0;             // BF16-MFMA variant: G_B staged in LDS (fits two workgroups per CU)
  int levels = 0;              // max order - 1
  std::vector<int> lvl_off;    // item offsets per level (levels + 1 entries; level l at index l-1)
  int n_meet = 0;
  LevelItem* d_items = nullptr;
  LevelItem* d_meet = nullptr;
  float* d_vbuf = nullptr;
  long* d_voff = nullptr;
  long* d_vcap = nullptr;
  float* d_one = nullptr;
  size_t lvl_lds = 0, meet_lds = 0;
  // graphs: one captured launch per output-pointer pair, at most kGraphs
  // kept; `done` is recorded after every replay, so an entry is destroyed
  // only once its last replay has finished
  struct GraphEntry {
    double* inner = nullptr;
    float* junc = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;
    uint64_t used = 0;
  };
  hipStream_t cap_stream = nullptr;
  std::vector<GraphEntry> graphs;
  uint64_t use_clock = 0;
};

namespace {

// dynamic LDS per workgroup: the CU's 160 KB split between co-resident
// workgroups, less room for the kernel's static LDS
const int kLdsBytes = 156 * 1024;
int lds_bytes_for(int per_cu) { return (160 * 1024) / per_cu - 4 * 1024; }

ttc_status check_pair_desc(const ttc_pair& p, int idx, uint32_t ops, ttc_dtype* dt) {
  const ttc_tt* ts[2] = {&p.x, &p.y};
  for (int s = 0; s < 2; ++s) {
    const ttc_tt* t = ts[s];
    const std::string nm = "pair " + std::to_string(idx) + (s ? " y" : " x");
    if (t->order < 2 || t->order > TTC_MAX_ORDER) return fail(TTC_ERR_SHAPE, nm + ": order outside [2, 32]");
    if (!t->modes || !t->ranks || !t->cores) return fail(TTC_ERR_NULL, nm + ": NULL descriptor array");
    if (t->dtype != TTC_F32 && t->dtype != TTC_BF16) return fail(TTC_ERR_DTYPE, nm + ": batched pairs are FP32 or BF16");
    if (t->ranks[0] != 1 || t->ranks[t->order] != 1) return fail(TTC_ERR_RANK, nm + ": boundary ranks must be 1");
    for (int k = 0; k < t->order; ++k) {
      if (t->modes[k] < 1 || t->ranks[k] < 1) return fail(TTC_ERR_SHAPE, nm + ": bad shape");
      if (t->ranks[k] > 128) return fail(TTC_ERR_UNSUPPORTED, nm + ": batched ranks are limited to 128");
      if (!t->cores[k]) return fail(TTC_ERR_NULL, nm + ": NULL core pointer");
      // core byte offsets are 32-bit in the kernels (row padding included)
      if (128.0 * t->modes[k] * 128.0 * 4.0 >= 2147483647.0)
        return fail(TTC_ERR_UNSUPPORTED, nm + ": batched mode sizes are limited to 32767");
    }
  }
  if (p.x.order != p.y.order) return fail(TTC_ERR_SHAPE, "pair " + std::to_string(idx) + ": orders differ");
  if (p.x.dtype != p.y.dtype) return fail(TTC_ERR_DTYPE, "pair " + std::to_string(idx) + ": dtypes differ");
  for (int k = 0; k < p.x.order; ++k)
    if (p.x.modes[k] != p.y.modes[k]) return fail(TTC_ERR_SHAPE, "pair " + std::to_string(idx) + ": modes differ");
  if ((ops & TTC_OP_SUFFIX2) && p.x.order < 3)
    return fail(TTC_ERR_SHAPE, "pair " + std::to_string(idx) + ": SUFFIX2 needs order >= 3");
  if (idx == 0) *dt = p.x.dtype;
  else if (*dt != p.x.dtype) return fail(TTC_ERR_DTYPE, "all pairs must share one dtype");
  return TTC_OK;
}

// Minimum-order FLOPs of one right-to-left step on core k.
double step_flops(const PairHost& p, int k) {
  const double I = p.modes[k], Rp = p.rx[k], Rn = p.rx[k + 1], Pp = p.ry[k], Pn = p.ry[k + 1];
  const double a = 2 * I * Rp * Pn * (Rn + Pp);
  const double b = 2 * I * Rn * Pp * (Pn + Rp);
  return std::min(a, b);
}

int pad16h(int n) { return (n + 15) & ~15; }

// Floats of one LDS interface buffer of the LDS-resident kernel for an
// R x P interface, in either layout (rows padded to 16, pitch padded + 4).
int lds_iface_elems_h(int R, int P) {
  return std::max(pad16h(P) * (pad16h(R) + 4), pad16h(R) * (pad16h(P) + 4));
}

// BF16 elements of one plane of the BF16-MFMA variant's interface (rows
// padded to 16, pitch padded + 8); its two planes take as many bytes as this
// many floats.
int lds16_iface_elems_h(int R, int P) {
  return std::max(pad16h(P) * (pad16h(R) + 8), pad16h(R) * (pad16h(P) + 8));
}

bool lds_mode(int mode) { return mode == 2 || mode == 3 || mode == 4; }

// A bound on the LDS-resident kernels' static LDS.
constexpr int kStaticLds = 1536;

int lds_variant(int mode) { return mode == 4 ? kBatchLdsB16 : mode == 3 ? kBatchLdsInPlace : kBatchLdsTwo; }

// Time model of the LDS-resident kernel for one pair, in shader cycles of
// one workgroup of four waves: per step a fixed cost (set-up, the first
// loads' latency, barriers), a cost per loop iteration of the busiest wave
// (the load latency one iteration of prefetch does not hide) and a cost
// per MFMA of that wave; the constants are a least-squares fit to per-step
// clocks of the 4096-pair workload.  Only used to order pairs (longest
// first) and to balance the static assignment.
double pair_time_model(const PairHost& h) {
  const int NW = 4;
  double t = 0;
  for (int k = h.order - 1; k >= 1; --k) {
    const int Rp = h.rx[k], Rn = h.rx[k + 1], Pp = h.ry[k], Pn = h.ry[k + 1], I = h.modes[k];
    const long cx = (long)pad16h(Rp) * pad16h(Pn) * (pad16h(Rn) + pad16h(Pp));
    const long cy = (long)pad16h(Pp) * pad16h(Rn) * (pad16h(Pn) + pad16h(Rp));
    const bool yf = cy < cx;
    const int Ma = yf ? Pp : Rp, Ka = yf ? Pn : Rn, Nb = yf ? Rp : Pp, Kb = yf ? Rn : Pn;
    const int RT = (Ma + 15) / 16, KC = (Ka + 15) / 16, PT = (Nb + 15) / 16, QT = (Kb + 15) / 16;
    int S = 1, best = ((RT + NW - 1) / NW) * I;
    for (int c = 2; c <= 2 * NW && c <= I && RT * c <= 2 * NW; c *= 2) {
      const int cost = ((RT * c + NW - 1) / NW) * ((I + c - 1) / c);
      if (cost < best) {
        best = cost;
        S = c;
      }
    }
    const double iters = (double)((RT * S + NW - 1) / NW) * ((I + S - 1) / S) * QT;
    t += 22000.0 + 1625.0 * iters + 46.0 * iters * 4 * (KC + PT);
  }
  return t + 10000.0;
}

// Per-pair sizes of one run: junction elements (R_{N-2} P_{N-2} with
// SUFFIX2), algorithmic FLOPs (the cheaper order of every right-to-left
// step, then the first cores' product and the final sum) and algorithmic
// bytes (every core read once, the FP64 scalar and the FP32 junction
// written once).
void pair_measures(const PairHost& h, uint32_t ops, size_t esz, int64_t* jlen, double* flops, double* bytes) {
  const int N = h.order;
  *jlen = (ops & TTC_OP_SUFFIX2) ? (int64_t)h.rx[N - 2] * h.ry[N - 2] : 0;
  double fl = 0, by = 0;
  for (int k = 1; k < N; ++k) fl += step_flops(h, k);
  fl += 2.0 * h.modes[0] * h.rx[1] * h.ry[1] + 2.0 * h.rx[1] * h.ry[1];
  for (int k = 0; k < N; ++k)
    by += (double)esz * ((double)h.rx[k] * h.modes[k] * h.rx[k + 1] + (double)h.ry[k] * h.modes[k] * h.ry[k + 1]);
  by += (ops & TTC_OP_INNER) ? 8.0 : 0.0;
  by += 4.0 * (double)*jlen;
  *flops = fl;
  *bytes = by;
}

PairHost host_pair(const ttc_pair& p) {
  PairHost h;
  const int N = p.x.order;
  h.order = N;
  h.modes.assign(p.x.modes, p.x.modes + N);
  h.rx.assign(p.x.ranks, p.x.ranks + N + 1);
  h.ry.assign(p.y.ranks, p.y.ranks + N + 1);
  h.xc.assign(p.x.cores, p.x.cores + N);
  h.yc.assign(p.y.cores, p.y.cores + N);
  return h;
}

// Pair indices by decreasing modelled cost, ties in index order: the order in
// which the LDS-resident kernels' workgroups claim pairs.
std::vector<int> longest_first(const std::vector<double>& cost) {
  std::vector<int> idx(cost.size());
  for (size_t i = 0; i < idx.size(); ++i) idx[i] = (int)i;
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return cost[a] > cost[b]; });
  return idx;
}

// Static longest-processing-time assignment: pairs sorted by cost, each
// given to the currently least-loaded workgroup.  Returns CSR lists.
void lpt_assign(const std::vector<double>& cost, int grid, std::vector<int>* begin, std::vector<int>* order) {
  const int n = (int)cost.size();
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return cost[a] > cost[b]; });
  typedef std::pair<double, int> Load;
  std::priority_queue<Load, std::vector<Load>, std::greater<Load>> heap;
  for (int g = 0; g < grid; ++g) heap.push(Load(0.0, g));
  std::vector<std::vector<int>> lists(grid);
  for (int i : idx) {
    Load l = heap.top();
    heap.pop();
    lists[l.second].push_back(i);
    l.first += cost[i];
    heap.push(l);
  }
  begin->assign(grid + 1, 0);
  order->clear();
  for (int g = 0; g < grid; ++g) {
    (*begin)[g] = (int)order->size();
    order->insert(order->end(), lists[g].begin(), lists[g].end());
  }
  (*begin)[grid] = (int)order->size();
}

BatchArgs make_args(ttc_plan* P, const int* begin, const int* order, double* inner, float* junc, int lds_elems,
                    int grid) {
  BatchArgs a;
  std::memset(&a, 0, sizeof(a));
  a.pairs = P->d_pairs;
  a.ipool = P->d_ipool;
  a.ppool = P->d_ppool;
  a.wg_begin = begin;
  a.order = order;
  a.ops = P->ops;
  a.lds_elems = lds_elems;
  a.iface = P->d_iface;
  a.iface_stride = 2 * P->max_rp;
  a.tbuf = P->d_tbuf;
  a.t_stride = P->max_t;
  a.inner = inner;
  a.junction = junc;
  a.buf_elems = P->buf_elems;
  a.stage = P->mode == 4 ? P->stage16 : 0;
  a.npairs = P->n;
  (void)grid;
  return a;
}

LevelArgs make_level_args(ttc_plan* P, double* inner, float* junc) {
  LevelArgs a;
  std::memset(&a, 0, sizeof(a));
  a.pairs = P->d_pairs;
  a.ipool = P->d_ipool;
  a.ppool = P->d_ppool;
  a.ops = P->ops;
  a.vbuf = P->d_vbuf;
  a.voff = P->d_voff;
  a.vcap = P->d_vcap;
  a.inner = inner;
  a.junction = junc;
  a.one = P->d_one;
  return a;
}

hipError_t run_levels(ttc_plan* P, double* inner, float* junc, hipStream_t s) {
  LevelArgs a = make_level_args(P, inner, junc);
  for (int l = 1; l <= P->levels; ++l) {
    a.level = l;
    a.items = P->d_items + P->lvl_off[l - 1];
    const int n = P->lvl_off[l] - P->lvl_off[l - 1];
    hipError_t e = launch_level(P->dt, a, n, P->lvl_lds, s);
    if (e != hipSuccess) return e;
  }
  if (P->ops & TTC_OP_INNER) {
    a.items = P->d_meet;
    return launch_meet_level(P->dt, a, P->n_meet, P->meet_lds, s);
  }
  return hipSuccess;
}

hipError_t run_persistent(ttc_plan* P, double* inner, float* junc, hipStream_t s) {
  BatchArgs a = make_args(P, P->d_begin, P->d_order, inner, junc, P->lds_elems, P->grid);
  return launch_batch(P->dt, a, P->grid, P->cfg.threads, s);
}

hipError_t run_lds(ttc_plan* P, double* inner, float* junc, hipStream_t s) {
  BatchArgs a = make_args(P, P->d_begin, P->d_order, inner, junc, P->lds_elems, P->grid);
  a.claim = P->d_claim;
  return launch_batch_lds(P->dt, a, P->grid, P->cfg.threads, lds_variant(P->mode), s);
}

hipError_t run_mode(ttc_plan* P, double* inner, float* junc, hipStream_t s) {
  if (P->mode == 1) return run_levels(P, inner, junc, s);
  if (lds_mode(P->mode)) return run_lds(P, inner, junc, s);
  return run_persistent(P, inner, junc, s);
}

// Largest number of LDS-resident workgroups per CU (bufs: interface buffers
// per workgroup).
int lds_kernel_per_cu(const ttc_plan* P, int bufs) {
  const int bytes = bufs * P->buf_elems * (int)sizeof(float) + 4 * 1024;
  return std::max(1, std::min(2, (160 * 1024) / bytes));
}

// The same for the BF16-MFMA variant: one interface buffer (two BF16 planes)
// and, when enabled, the G_B stage.
int lds16_kernel_per_cu(const ttc_plan* P) {
  const int bytes = P->buf_elems * (int)sizeof(float) + (P->stage16 ? kBatchStageBytes : 0) + kStaticLds;
  return std::max(1, std::min(2, (160 * 1024) / bytes));
}

ttc_status upload_assignment(ttc_plan* P, const LaunchCfg& c, int* grid_out, int* lds_out) {
  const int grid = std::min(P->cus * c.per_cu, std::max(P->n, 1));
  std::vector<int> begin, order;
  lpt_assign(P->cost, grid, &begin, &order);
  if (lds_mode(c.mode)) order = longest_first(P->cost);  // claimed one by one at run time
  TTC_HIP(hipMemcpy(P->d_begin, begin.data(), begin.size() * sizeof(int), hipMemcpyHostToDevice));
  TTC_HIP(hipMemcpy(P->d_order, order.data(), order.size() * sizeof(int), hipMemcpyHostToDevice));
  *grid_out = grid;
  *lds_out = lds_bytes_for(c.per_cu) / (int)sizeof(float);
  return TTC_OK;
}

std::string cache_key(const ttc_plan* P) {
  uint64_t h = 1469598103934665603ULL;
  auto mix = [&](uint64_t v) {
    h ^= v;
    h *= 1099511628211ULL;
  };
  for (const PairHost& p : P->pairs) {
    mix(p.order);
    for (int v : p.modes) mix(v);
    for (int v : p.rx) mix(v);
    for (int v : p.ry) mix(v);
  }
  mix(P->ops);
  mix(P->dt);
  mix(P->prec);
  std::ostringstream os;
  os << "gfx950|abi" << TTC_ABI_VERSION << "|s5|" << std::hex << h;
  return os.str();
}

// Tiny persistent cache: one "key mode threads per_cu" line per entry.
std::mutex g_cache_mu;
bool cache_lookup(const std::string& key, LaunchCfg* c) {
  const char* path = std::getenv("TTC_AUTOTUNE_CACHE");
  if (!path) return false;
  std::lock_guard<std::mutex> lk(g_cache_mu);
  std::ifstream f(path);
  std::string k;
  int m, t, pc;
  while (f >> k >> m >> t >> pc)
    if (k == key) {
      c->mode = m;
      c->threads = t;
      c->per_cu = pc;
      return true;
    }
  return false;
}
void cache_store(const std::string& key, const LaunchCfg& c) {
  const char* path = std::getenv("TTC_AUTOTUNE_CACHE");
  if (!path) return;
  std::lock_guard<std::mutex> lk(g_cache_mu);
  std::ofstream f(path, std::ios::app);
  f << key << " " << c.mode << " " << c.threads << " " << c.per_cu << "\n";
}

ttc_status autotune(ttc_plan* P) {
  const std::string key = cache_key(P);
  const char* forced = std::getenv("TTC_BATCH_MODE");  // testing: levels | persistent | lds | lds1 | lds1b
  int want = -1;
  if (forced) {
    if (std::strcmp(forced, "persistent") == 0) want = 0;
    if (std::strcmp(forced, "levels") == 0) want = 1;
    if (std::strcmp(forced, "lds") == 0) want = 2;
    if (std::strcmp(forced, "lds1") == 0) want = 3;
    if (std::strcmp(forced, "lds1b") == 0) want = 4;
    // the BF16-MFMA variant takes BF16 cores only; FP32 plans keep the tuner's choice
    if (want == 4 && P->dt != TTC_BF16) want = -1;
  }
  // the plan's precision: BF16 keeps only the BF16-MFMA schedule, F32 every
  // schedule but that one
  if (P->prec == TTC_PREC_BF16) want = 4;
  if (P->prec == TTC_PREC_F32 && want == 4) want = -1;
  const bool no16 = P->prec == TTC_PREC_F32;
  LaunchCfg best;
  if (cache_lookup(key, &best) && (want < 0 || want == best.mode) && !(no16 && best.mode == 4)) {
    P->mode = best.mode;
    P->cfg = best;
    return upload_assignment(P, best, &P->grid, &P->lds_elems);
  }
  std::vector<LaunchCfg> cands;
  if (P->dt == TTC_BF16 && !no16 && (want < 0 || want == 4))
    for (int pc = 1; pc <= lds16_kernel_per_cu(P); ++pc) cands.push_back({4, 256, pc});
  if (want < 0 || want == 3)
    for (int pc = 1; pc <= lds_kernel_per_cu(P, 1); ++pc) cands.push_back({3, 256, pc});
  if (want < 0 || want == 2) {
    for (int pc = 1; pc <= lds_kernel_per_cu(P, 2); ++pc) {
      cands.push_back({2, 256, pc});
      cands.push_back({2, 512, pc});
    }
  }
  if (want < 0 || want == 0) {
    cands.push_back({0, 512, 1});
    cands.push_back({0, 256, 1});
    cands.push_back({0, 512, 2});
    cands.push_back({0, 256, 2});
  }
  if (want < 0 || want == 1) cands.push_back({1, 256, 1});
  if (cands.empty()) return fail(TTC_ERR_UNSUPPORTED, "no schedule of the plan's precision fits these pairs");
  double* d_inner = nullptr;
  float* d_junc = nullptr;
  TTC_HIP(hipMalloc(&d_inner, sizeof(double) * std::max(P->n, 1)));
  TTC_HIP(hipMalloc(&d_junc, sizeof(float) * std::max<int64_t>(P->joff.back(), 1)));
  hipEvent_t e0, e1;
  TTC_HIP(hipEventCreate(&e0));
  TTC_HIP(hipEventCreate(&e1));
  float best_ms = 1e30f;
  for (const LaunchCfg& c : cands) {
    P->mode = c.mode;
    P->cfg = c;
    TTC_TRY(upload_assignment(P, c, &P->grid, &P->lds_elems));
    TTC_HIP(run_mode(P, d_inner, d_junc, 0));
    TTC_HIP(hipEventRecord(e0, 0));
    for (int r = 0; r < 2; ++r) TTC_HIP(run_mode(P, d_inner, d_junc, 0));
    TTC_HIP(hipEventRecord(e1, 0));
    TTC_HIP(hipEventSynchronize(e1));
    float ms = 0;
    TTC_HIP(hipEventElapsedTime(&ms, e0, e1));
    if (ms < best_ms) {
      best_ms = ms;
      best = c;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(d_inner);
  (void)hipFree(d_junc);
  P->mode = best.mode;
  P->cfg = best;
  if (!forced) cache_store(key, best);
  return upload_assignment(P, best, &P->grid, &P->lds_elems);
}

void destroy_graph(ttc_plan::GraphEntry& g) {
  if (g.done) (void)hipEventSynchronize(g.done);
  if (g.exec) (void)hipGraphExecDestroy(g.exec);
  if (g.graph) (void)hipGraphDestroy(g.graph);
  if (g.done) (void)hipEventDestroy(g.done);
  g = ttc_plan::GraphEntry();
}

const size_t kGraphs = 4;

// The graph entry that replays the plan's launch into (d_inner,
// d_junction): found, or captured on the plan's own stream (thread-local
// capture, so other threads' work is not captured), evicting the least
// recently used entry after its last replay has finished.
ttc_status graph_for(ttc_plan* P, double* d_inner, float* d_junction, ttc_plan::GraphEntry** out) {
  for (auto& g : P->graphs)
    if (g.inner == d_inner && g.junc == d_junction) {
      g.used = ++P->use_clock;
      *out = &g;
      return TTC_OK;
    }
  if (P->graphs.size() >= kGraphs) {
    size_t lru = 0;
    for (size_t i = 1; i < P->graphs.size(); ++i)
      if (P->graphs[i].used < P->graphs[lru].used) lru = i;
    destroy_graph(P->graphs[lru]);
    P->graphs.erase(P->graphs.begin() + lru);
  }
  if (!P->cap_stream) TTC_HIP(hipStreamCreateWithFlags(&P->cap_stream, hipStreamNonBlocking));
  ttc_plan::GraphEntry g;
  TTC_HIP(hipStreamBeginCapture(P->cap_stream, hipStreamCaptureModeThreadLocal));
  hipError_t le = run_mode(P, d_inner, d_junction, P->cap_stream);
  hipError_t ce = hipStreamEndCapture(P->cap_stream, &g.graph);
  if (le != hipSuccess || ce != hipSuccess) {
    if (g.graph) (void)hipGraphDestroy(g.graph);
    return fail(TTC_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(le != hipSuccess ? le : ce));
  }
  hipError_t ie = hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0);
  if (ie == hipSuccess) ie = hipEventCreateWithFlags(&g.done, hipEventDisableTiming);
  if (ie != hipSuccess) {
    destroy_graph(g);
    return fail(TTC_ERR_HIP, std::string("graph instantiate: ") + hipGetErrorString(ie));
  }
  g.inner = d_inner;
  g.junc = d_junction;
  g.used = ++P->use_clock;
  P->graphs.push_back(g);
  *out = &P->graphs.back();
  return TTC_OK;
}

void release(ttc_plan* P) {
  for (auto& g : P->graphs) destroy_graph(g);
  P->graphs.clear();
  if (P->cap_stream) (void)hipStreamDestroy(P->cap_stream);
  if (P->dmem) (void)hipFree(P->dmem);
  if (P->dmem_levels) (void)hipFree(P->dmem_levels);
  P->dmem_levels = nullptr;
  P->cap_stream = nullptr;
  P->dmem = nullptr;
}

}  // namespace

extern "C" {

ttc_status tt_batch_plan_create(const ttc_pair* pairs, int32_t n, uint32_t ops, ttc_prec prec, ttc_plan** plan) {
  if (!plan) return fail(TTC_ERR_NULL, "plan is NULL");
  *plan = nullptr;
  if (!pairs || n < 1) return fail(TTC_ERR_NULL, "no pairs");
  if (ops == 0 || (ops & ~(TTC_OP_INNER | TTC_OP_SUFFIX2))) return fail(TTC_ERR_UNSUPPORTED, "bad ops mask");
  if (prec != TTC_PREC_AUTO && prec != TTC_PREC_F32 && prec != TTC_PREC_BF16)
    return fail(TTC_ERR_UNSUPPORTED, "batched precision is AUTO, F32 or BF16");
  ttc_dtype dt = TTC_F32;
  for (int i = 0; i < n; ++i) TTC_TRY(check_pair_desc(pairs[i], i, ops, &dt));
  if (prec == TTC_PREC_BF16 && dt != TTC_BF16)
    return fail(TTC_ERR_UNSUPPORTED, "BF16 precision needs BF16 cores (the BF16-MFMA steps)");
  ttc_plan* P = new ttc_plan();
  P->n = n;
  P->ops = ops;
  P->dt = dt;
  P->prec = prec;
  P->buf_elems = 16 * (16 + 4);  // V_N = [1] padded
  const size_t esz = dt == TTC_BF16 ? 2 : 4;
  P->pairs.resize(n);
  P->joff.assign(n + 1, 0);
  P->cost.assign(n, 0.0);
  std::vector<PairDev> pd(n);
  std::vector<int> ipool;
  std::vector<void*> ppool;
  for (int i = 0; i < n; ++i) {
    PairHost& h = P->pairs[i];
    const ttc_tt& x = pairs[i].x;
    const ttc_tt& y = pairs[i].y;
    const int N = x.order;
    h.order = N;
    h.modes.assign(x.modes, x.modes + N);
    h.rx.assign(x.ranks, x.ranks + N + 1);
    h.ry.assign(y.ranks, y.ranks + N + 1);
    h.xc.assign(x.cores, x.cores + N);
    h.yc.assign(y.cores, y.cores + N);
    pd[i].order = N;
    pd[i].ibase = (int)ipool.size();
    pd[i].pbase = (int)ppool.size();
    pd[i].pad = 0;
    pd[i].jout = P->joff[i];
    ipool.insert(ipool.end(), h.modes.begin(), h.modes.end());
    ipool.insert(ipool.end(), h.rx.begin(), h.rx.end());
    ipool.insert(ipool.end(), h.ry.begin(), h.ry.end());
    ppool.insert(ppool.end(), h.xc.begin(), h.xc.end());
    ppool.insert(ppool.end(), h.yc.begin(), h.yc.end());
    int64_t jlen = 0;
    double fl = 0, by = 0;
    pair_measures(h, ops, esz, &jlen, &fl, &by);
    P->joff[i + 1] = P->joff[i] + jlen;
    P->flops += fl;
    P->bytes += by;
    P->cost[i] = pair_time_model(h);
    for (int b = 1; b <= N; ++b) P->max_rp = std::max<long>(P->max_rp, (long)h.rx[b] * ((h.ry[b] & 1) ? h.ry[b] : h.ry[b] + 1));
    for (int b = 1; b <= N; ++b) {
      P->buf_elems = std::max(P->buf_elems, lds_iface_elems_h(h.rx[b], h.ry[b]));
      if (dt == TTC_BF16) P->buf_elems = std::max(P->buf_elems, lds16_iface_elems_h(h.rx[b], h.ry[b]));
    }
  }
  P->buf_elems = (P->buf_elems + 7) & ~7;  // BF16 lo plane at a 16-byte boundary
  // the BF16-MFMA variant stages G_B in LDS when two workgroups per CU still fit
  P->stage16 = (dt == TTC_BF16 && 2 * (P->buf_elems * 4 + kBatchStageBytes + kStaticLds) <= 160 * 1024) ? 1 : 0;
  hipError_t e = hipGetDevice(&P->device);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&P->cus, hipDeviceAttributeMultiprocessorCount, P->device);
  if (e != hipSuccess) {
    delete P;
    return fail(TTC_ERR_HIP, std::string("device query: ") + hipGetErrorString(e));
  }
  P->max_grid = P->cus * 2;
  // one device allocation for every table
  auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
  size_t off = 0;
  const size_t o_pairs = off;
  off += al(sizeof(PairDev) * n);
  const size_t o_ipool = off;
  off += al(sizeof(int) * ipool.size());
  const size_t o_ppool = off;
  off += al(sizeof(void*) * ppool.size());
  const size_t o_begin = off;
  off += al(sizeof(int) * (P->max_grid + 1));
  const size_t o_order = off;
  off += al(sizeof(int) * n);
  const size_t o_ident = off;
  off += al(sizeof(int) * n);
  const size_t o_01 = off;
  off += al(sizeof(int) * 2);
  const size_t o_claim = off;
  off += al(sizeof(int) * 2);
  const size_t o_iface = off;
  off += al(sizeof(float) * 2 * P->max_rp * P->max_grid);
  const size_t o_tbuf = off;
  off += al(sizeof(float) * P->max_t * P->max_grid);
  e = hipMalloc(&P->dmem, off);
  if (e != hipSuccess) {
    delete P;
    return fail(TTC_ERR_HIP, std::string("plan allocation: ") + hipGetErrorString(e));
  }
  char* base = (char*)P->dmem;
  P->d_pairs = (PairDev*)(base + o_pairs);
  P->d_ipool = (int*)(base + o_ipool);
  P->d_ppool = (void**)(base + o_ppool);
  P->d_begin = (int*)(base + o_begin);
  P->d_order = (int*)(base + o_order);
  P->d_ident = (int*)(base + o_ident);
  P->d_01 = (int*)(base + o_01);
  P->d_claim = (int*)(base + o_claim);
  P->d_iface = (float*)(base + o_iface);
  P->d_tbuf = (float*)(base + o_tbuf);
  std::vector<int> ident(n);
  for (int i = 0; i < n; ++i) ident[i] = i;
  const int zo[2] = {0, 1}, zz[2] = {0, 0};
  ttc_status st = TTC_OK;
  auto cp = [&](void* dst, const void* src, size_t b) {
    if (st == TTC_OK && b) {
      hipError_t ee = hipMemcpy(dst, src, b, hipMemcpyHostToDevice);
      if (ee != hipSuccess) st = fail(TTC_ERR_HIP, std::string("descriptor upload: ") + hipGetErrorString(ee));
    }
  };
  cp(P->d_pairs, pd.data(), sizeof(PairDev) * n);
  cp(P->d_ipool, ipool.data(), sizeof(int) * ipool.size());
  cp(P->d_ppool, ppool.data(), sizeof(void*) * ppool.size());
  cp(P->d_ident, ident.data(), sizeof(int) * n);
  cp(P->d_01, zo, sizeof(zo));
  cp(P->d_claim, zz, sizeof(zz));
  if (st == TTC_OK) {
    hipError_t ee = batch_set_lds(kLdsBytes);
    if (ee == hipSuccess) ee = batch_lds_set_lds(2 * P->buf_elems * (int)sizeof(float), P->stage16 ? kBatchStageBytes : 0);
    if (ee != hipSuccess) st = fail(TTC_ERR_HIP, std::string("kernel attribute: ") + hipGetErrorString(ee));
  }
  // level-by-level tables: items (pair, 16-row tile) of every level, heavy first
  if (st == TTC_OK) {
    int maxN = 0;
    for (const PairHost& h : P->pairs) maxN = std::max(maxN, h.order);
    P->levels = maxN - 1;
    std::vector<LevelItem> items;
    P->lvl_off.assign(1, 0);
    for (int l = 1; l <= P->levels; ++l) {
      std::vector<std::pair<double, LevelItem>> lv;
      for (int q = 0; q < n; ++q) {
        const PairHost& h = P->pairs[q];
        const int k = h.order - l;
        if (k < 1) continue;
        const int RT = (h.rx[k] + 15) / 16;
        const double c = (double)h.modes[k] * ((h.ry[k + 1] + 15) / 16) *
                         ((h.rx[k + 1] + 15) / 16 + (h.ry[k] + 15) / 16);
        for (int rt = 0; rt < RT; ++rt) lv.push_back({c, LevelItem{q, rt}});
      }
      std::stable_sort(lv.begin(), lv.end(), [](const std::pair<double, LevelItem>& a,
                                                const std::pair<double, LevelItem>& b) { return a.first > b.first; });
      for (auto& e : lv) items.push_back(e.second);
      P->lvl_off.push_back((int)items.size());
    }
    std::vector<LevelItem> meet;
    for (int q = 0; q < n; ++q) meet.push_back(LevelItem{q, 0});
    P->n_meet = n;
    std::vector<long> voff(n), vcap(n);
    long vtot = 0;
    int maxP = 1, maxW1 = 1;
    for (int q = 0; q < n; ++q) {
      const PairHost& h = P->pairs[q];
      long cap = 1;
      for (int b = 1; b < h.order; ++b) cap = std::max(cap, (long)h.rx[b] * h.ry[b]);
      for (int b = 1; b <= h.order; ++b) maxP = std::max(maxP, h.ry[b]);
      maxW1 = std::max(maxW1, h.rx[1] * h.ry[1]);
      cap = (cap + 3) & ~3L;
      voff[q] = vtot;
      vcap[q] = cap;
      vtot += 2 * cap;
    }
    P->lvl_lds = (size_t)4 * 16 * maxP * sizeof(float);
    P->meet_lds = (size_t)maxW1 * sizeof(float);
    void* lm = nullptr;
    const size_t b_items = al(sizeof(LevelItem) * std::max<size_t>(items.size(), 1));
    const size_t b_meet = al(sizeof(LevelItem) * n);
    const size_t b_off = al(sizeof(long) * n);
    const size_t b_v = al(sizeof(float) * vtot);
    hipError_t ee = hipMalloc(&lm, b_items + b_meet + 2 * b_off + b_v + 256);
    if (ee != hipSuccess) {
      st = fail(TTC_ERR_HIP, std::string("plan allocation: ") + hipGetErrorString(ee));
    } else {
      P->dmem_levels = lm;
      char* c = (char*)lm;
      P->d_items = (LevelItem*)c;
      P->d_meet = (LevelItem*)(c + b_items);
      P->d_voff = (long*)(c + b_items + b_meet);
      P->d_vcap = (long*)(c + b_items + b_meet + b_off);
      P->d_vbuf = (float*)(c + b_items + b_meet + 2 * b_off);
      P->d_one = (float*)(c + b_items + b_meet + 2 * b_off + b_v);
      const float one = 1.f;
      cp(P->d_one, &one, sizeof(float));
      cp(P->d_items, items.data(), sizeof(LevelItem) * items.size());
      cp(P->d_meet, meet.data(), sizeof(LevelItem) * n);
      cp(P->d_voff, voff.data(), sizeof(long) * n);
      cp(P->d_vcap, vcap.data(), sizeof(long) * n);
    }
    if (st == TTC_OK) {
      ee = level_set_lds((int)P->lvl_lds, (int)P->meet_lds);
      if (ee != hipSuccess) st = fail(TTC_ERR_HIP, std::string("kernel attribute: ") + hipGetErrorString(ee));
    }
  }
  if (st == TTC_OK) st = autotune(P);
  if (st == TTC_OK) {
    hipError_t ee = hipDeviceSynchronize();
    if (ee != hipSuccess) st = fail(TTC_ERR_HIP, std::string("plan setup: ") + hipGetErrorString(ee));
  }
  if (st != TTC_OK) {
    release(P);
    delete P;
    return st;
  }
  *plan = P;
  return TTC_OK;
}

ttc_status tt_batch_plan_query(const ttc_pair* pairs, int32_t n, uint32_t ops, int64_t* junction_offsets,
                               double* flops, double* bytes, double* cost, int32_t* claim_order) {
  if (!pairs || n < 1) return fail(TTC_ERR_NULL, "no pairs");
  if (ops == 0 || (ops & ~(TTC_OP_INNER | TTC_OP_SUFFIX2))) return fail(TTC_ERR_UNSUPPORTED, "bad ops mask");
  ttc_dtype dt = TTC_F32;
  for (int i = 0; i < n; ++i) TTC_TRY(check_pair_desc(pairs[i], i, ops, &dt));
  const size_t esz = dt == TTC_BF16 ? 2 : 4;
  std::vector<double> c(n);
  int64_t off = 0;
  double tf = 0, tb = 0;
  if (junction_offsets) junction_offsets[0] = 0;
  for (int i = 0; i < n; ++i) {
    const PairHost h = host_pair(pairs[i]);
    int64_t jlen = 0;
    double fl = 0, by = 0;
    pair_measures(h, ops, esz, &jlen, &fl, &by);
    off += jlen;
    tf += fl;
    tb += by;
    c[i] = pair_time_model(h);
    if (junction_offsets) junction_offsets[i + 1] = off;
    if (cost) cost[i] = c[i];
  }
  if (flops) *flops = tf;
  if (bytes) *bytes = tb;
  if (claim_order) {
    const std::vector<int> idx = longest_first(c);
    for (int i = 0; i < n; ++i) claim_order[i] = idx[i];
  }
  return TTC_OK;
}

ttc_status tt_batch_plan_info(const ttc_plan* P, int64_t* junction_offsets, double* flops, double* bytes) {
  if (!P) return fail(TTC_ERR_NULL, "plan is NULL");
  if (junction_offsets) std::memcpy(junction_offsets, P->joff.data(), sizeof(int64_t) * (P->n + 1));
  if (flops) *flops = P->flops;
  if (bytes) *bytes = P->bytes;
  return TTC_OK;
}

ttc_status tt_batch_plan_config(const ttc_plan* P, int32_t* mode, int32_t* threads, int32_t* wg_per_cu) {
  if (!P) return fail(TTC_ERR_NULL, "plan is NULL");
  if (mode) *mode = P->mode;
  if (threads) *threads = P->cfg.threads;
  if (wg_per_cu) *wg_per_cu = P->cfg.per_cu;
  return TTC_OK;
}

ttc_status tt_batch_run(ttc_plan* P, double* d_inner, float* d_junction, void* stream) {
  if (!P) return fail(TTC_ERR_NULL, "plan is NULL");
  if ((P->ops & TTC_OP_INNER) && !d_inner) return fail(TTC_ERR_NULL, "d_inner is NULL");
  if ((P->ops & TTC_OP_SUFFIX2) && !d_junction) return fail(TTC_ERR_NULL, "d_junction is NULL");
  hipStream_t s = (hipStream_t)stream;
  ttc_plan::GraphEntry* g = nullptr;
  TTC_TRY(graph_for(P, d_inner, d_junction, &g));
  TTC_HIP(hipGraphLaunch(g->exec, s));
  TTC_HIP(hipEventRecord(g->done, s));
  return TTC_OK;
}

ttc_status tt_batch_run_traced(ttc_plan* P, double* d_inner, float* d_junction, int64_t* d_clock, void* stream) {
  if (!P) return fail(TTC_ERR_NULL, "plan is NULL");
  if ((P->ops & TTC_OP_INNER) && !d_inner) return fail(TTC_ERR_NULL, "d_inner is NULL");
  if ((P->ops & TTC_OP_SUFFIX2) && !d_junction) return fail(TTC_ERR_NULL, "d_junction is NULL");
  if (!d_clock) return fail(TTC_ERR_NULL, "d_clock is NULL");
  if (!lds_mode(P->mode)) return fail(TTC_ERR_UNSUPPORTED, "tracing needs an LDS-resident schedule");
  BatchArgs a = make_args(P, P->d_begin, P->d_order, d_inner, d_junction, P->lds_elems, P->grid);
  a.clock = reinterpret_cast<long long*>(d_clock);
  a.claim = P->d_claim;
  TTC_HIP(launch_batch_lds(P->dt, a, P->grid, P->cfg.threads, lds_variant(P->mode), (hipStream_t)stream));
  return TTC_OK;
}

ttc_status tt_batch_run_plain(ttc_plan* P, double* d_inner, float* d_junction, void* stream) {
  if (!P) return fail(TTC_ERR_NULL, "plan is NULL");
  if ((P->ops & TTC_OP_INNER) && !d_inner) return fail(TTC_ERR_NULL, "d_inner is NULL");
  if ((P->ops & TTC_OP_SUFFIX2) && !d_junction) return fail(TTC_ERR_NULL, "d_junction is NULL");
  hipStream_t s = (hipStream_t)stream;
  // one launch per pair of the LDS-resident kernel (one workgroup each)
  for (int p = 0; p < P->n; ++p) {
    BatchArgs a = make_args(P, P->d_01, P->d_ident + p, d_inner, d_junction, 0, 1);
    TTC_HIP(launch_batch_lds(P->dt, a, 1, 256, kBatchLdsTwo, s));
  }
  return TTC_OK;
}

void tt_batch_plan_destroy(ttc_plan* P) {
  if (!P) return;
  (void)hipDeviceSynchronize();
  release(P);
  delete P;
}

}  // extern "C"
