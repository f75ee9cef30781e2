// Internal interface between the host runtime (validation, planning,
// dispatch) and the kernel launchers.  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>

#include "../../include/ttc.h"

namespace ttc {

// Runs set() the first time it is reached with a given device current and
// again only after a failure: a kernel's dynamic-LDS limit is a setting of
// each device.  Two threads arriving together may both run set(), which only
// repeats the same attribute write.
constexpr int kMaxDevices = 64;
template <typename F>
hipError_t once_per_device(std::atomic<bool> (&done)[kMaxDevices], F&& set) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return set();
  if (done[dev].load(std::memory_order_acquire)) return hipSuccess;
  e = set();
  if (e == hipSuccess) done[dev].store(true, std::memory_order_release);
  return e;
}

// TT descriptor passed by value to kernels (device core pointers).
struct TTDev {
  int order;
  int modes[TTC_MAX_ORDER];
  int ranks[TTC_MAX_ORDER + 1];
  const void* cores[TTC_MAX_ORDER];
};

// ---------------------------------------------------------------- sweeps
// Block b runs direction dir[b] (0: left to right, 1: right to left,
// -1: idle) up to bond stop[b] and stores the final interface (row-major
// R x P, compute type) at out[b].
struct SweepArgs {
  TTDev x, y;
  int dir[2];
  int stop[2];
  void* out[2];
  int max_rp;      // interface buffer capacity (elements)
  int tcap;        // capacity of the per-mode intermediate (elements)
  void* t_global;  // intermediate in global memory (null: in LDS)
  long t_stride;   // elements per block in t_global
  void* i_global;  // the two interface buffers in global memory (null: in LDS)
  long i_stride;   // elements per block in i_global (2 * max_rp)
  int chain;       // chained-MFMA steps (ranks <= 128; odd-pitch interfaces)
};

// Left/right checkpoints for the inner-product gradient (phase A) and the
// per-segment gradient pass (phase B).
struct GradArgs {
  TTDev x, y;
  int stride;       // checkpoint stride c
  int nseg;         // ceil(N / c)
  void* ckW;        // nseg x max_rp: W_{s c}
  void* ckV;        // nseg x max_rp: V_{min((s+1)c, N)}
  void* segV;       // nseg x c x max_rp: V_{k+1} for k in segment s (slot k)
  void* segW;       // nseg x c x max_rp: W_k for k in segment s (slot k)
  void* g_global;   // per-block product buffers of the gradient kernel (null: LDS)
  long g_stride;    // elements per block in g_global
  void* dx[TTC_MAX_ORDER];
  void* dy[TTC_MAX_ORDER];
  const double* gz;
  int max_rp;
  int tcap;
  void* t_global;
  long t_stride;
  void* i_global;
  long i_stride;
};

// Natural-order lift of a junction matrix K (see tt_contract_modes).
// LIFT_ABSORB_M and LIFT_DELTA_SPLIT serve contractions whose junction has
// four bonds, T[(a, g), (b, d)] (row-major a, g, b, d; sizes r0 of the core
// for b, kg for g, kd for d), carried as q = g * kd + d (Q = kg * kd).
enum LiftOp {
  LIFT_COPY = 0,
  LIFT_ABSORB_L = 1,
  LIFT_ABSORB_R = 2,
  LIFT_DELTA = 3,
  LIFT_DELTA_LAST = 4,
  LIFT_ABSORB_M = 5,     // dst (ka, n, r1 * Q): sum_b T[(a, g), (b, d)] G[b, i, s]
  LIFT_DELTA_SPLIT = 6   // dst (r0 * Q, n, kd): G[y, i, g] if d == d', src r1 = kg
};
// Unsigned division by a run-time invariant d with one multiply-high
// (Granlund and Montgomery, "Division by invariant integers using
// multiplication", 1994, sec. 4): with l = ceil(log2 d) and
// m = floor(2^32 (2^l - d) / d) + 1, floor(x / d) = (mulhi(m, x) + x) >> l
// for every 32-bit x.
struct FastDiv {
  uint32_t m, l;
};
inline FastDiv make_fastdiv(uint32_t d) {
  FastDiv f;
  uint32_t l = 0;
  while (l < 32 && ((uint64_t)1 << l) < d) ++l;
  f.l = l;
  f.m = (uint32_t)((((uint64_t)1 << 32) * (((uint64_t)1 << l) - d)) / d + 1);
  return f;
}

struct LiftCore {
  int op;
  int r0, n, r1;     // source core shape
  int d0, d1;        // destination bond sizes (n is shared)
  int kg, kd;        // LIFT_ABSORB_M / LIFT_DELTA_SPLIT: the carried bond's two factors
  const void* src;
  void* dst;
  // filled by launch_lift: the core's items (runs of `vec` consecutive
  // outputs of one line, w per line), numbered from item_begin (a multiple
  // of 64, so a wave's items lie in one core)
  long item_begin, items;
  int vec, w;
  FastDiv fw, fn;
};
#define TTC_MAX_LIFT (2 * TTC_MAX_ORDER)
struct LiftArgs {
  int ncores;
  int Q;             // columns of K
  int kr;            // rows of K
  const void* K;     // compute type
  FastDiv fq;        // filled by launch_lift
  LiftCore c[TTC_MAX_LIFT];
};

struct DenseArgs {
  TTDev t;           // compute-type cores
  long numel;
  void* out;
};

// Mode-n products: one entry per listed mode.
struct ModeNEntry {
  int r0, I, r1, J;
  long first;        // first output element of this entry (global numbering)
  const void* src;
  const void* A;
  void* dst;
};
struct ModeNArgs {
  int count;
  long total;
  ModeNEntry e[TTC_MAX_ORDER];
};

// TT-matrix x TT-vector, one entry per core.
struct MpoCore {
  int a0, I, J, a1;  // MPO core shape
  int r0, r1;        // TT-vector core bonds
  int blk_begin;     // first workgroup of this core
  const void* w;
  const void* v;
  void* out;
};
struct MpoArgs {
  int ncores;
  int nblk;
  MpoCore c[TTC_MAX_ORDER];
};

// ------------------------------------------------- single-pair LDS sweeps
// One workgroup per side; a side sweeps its pair right to left from
// V_order = [1] down to V_stop with the LDS-resident step (FP32 or BF16
// cores, ranks <= 128), and stores
//   out:   V_stop, row-major R x P (FP32), when set;
//   all:   every V_k, k = order .. max(stop, 1), row-major, at
//          all + (slot_a * k + slot_b) * all_stride, when set;
//   inner: with stop = 1, <X, Y> (FP64) finished with the first cores.
// A left-to-right sweep is the right-to-left sweep of the reversed pair
// whose cores have their two rank axes exchanged (see launch_core_reverse):
// its V'_j is W_{order - j}, in the same orientation.
struct PairLdsSide {
  TTDev x, y;
  int stop;
  float* out;
  float* all;
  int slot_a, slot_b;
  long all_stride;
  double* inner;
};
struct PairLdsArgs {
  PairLdsSide side[2];
  bool m16;  // BF16 cores on BF16 MFMA (interface as BF16 hi / lo planes)
  int lo;    // set by launch_pair_lds: elements of one plane (m16)
};
// True when the LDS-resident sweep handles the pair (FP32/BF16, ranks <= 128).
bool pair_lds_ok(const TTDev& x, const TTDev& y);
hipError_t launch_pair_lds(ttc_dtype dt, const PairLdsArgs& a, int nsides, hipStream_t s);

// dst core j of each list = src core n-1-j with its rank axes exchanged:
// (R, I, R1) -> (R1, I, R).  esz: element bytes (2 or 4).
struct CoreRevItem {
  const void* src;
  void* dst;
  int R, I, R1;
};
struct CoreRevArgs {
  int n;
  int esz;
  CoreRevItem c[2 * TTC_MAX_ORDER];
};
hipError_t launch_core_reverse(const CoreRevArgs& a, hipStream_t s);

// launchers (return the launch status)
hipError_t launch_sweep(ttc_dtype dt, const SweepArgs& a, int nblocks, size_t lds, hipStream_t s);
hipError_t launch_meet(ttc_dtype dt, const void* W, const void* V, int n, double* out, hipStream_t s);
hipError_t launch_grad_ckpt(ttc_dtype dt, const GradArgs& a, size_t lds, hipStream_t s);
hipError_t launch_grad_seg(ttc_dtype dt, const GradArgs& a, size_t lds, hipStream_t s);
// One workgroup per (X or Y, core, mode index): the gradient slice from the
// stored interfaces.  lds: bytes of its product buffer (0 with g_global).
hipError_t launch_grad_core(ttc_dtype dt, const GradArgs& a, int blocks, size_t lds, hipStream_t s);
hipError_t launch_lift(ttc_dtype dt, const LiftArgs& a, int total_lines, hipStream_t s);
hipError_t launch_dense(bool f64, const DenseArgs& a, hipStream_t s);
hipError_t launch_mode_n(ttc_dtype dt, const ModeNArgs& a, hipStream_t s);
hipError_t launch_mpo(ttc_dtype dt, bool bf16_mfma, const MpoArgs& a, hipStream_t s);
hipError_t sweep_set_lds_limits();

int lds_limit_bytes();

}  // namespace ttc
