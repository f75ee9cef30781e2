// Internal interface of the batched persistent sweep.
#pragma once
#include <hip/hip_runtime.h>

#include "ttc_internal.h"

namespace ttc {

struct PairDev {
  int order;
  int ibase;   // modes[N], ranks_x[N+1], ranks_y[N+1] at ipool + ibase
  int pbase;   // x cores[N], y cores[N] at ppool + pbase
  int pad;
  long jout;   // junction offset (elements)
};

struct BatchArgs {
  const PairDev* pairs;
  const int* ipool;
  const void* const* ppool;
  const int* wg_begin;   // [grid + 1]: slice of `order` owned by each workgroup
  const int* order;      // pair indices
  unsigned ops;
  int lds_elems;         // FP32 elements of dynamic LDS per workgroup
  void* iface;           // per-workgroup interface slices (FP32)
  long iface_stride;
  void* tbuf;            // per-workgroup intermediate slices (FP32)
  long t_stride;
  double* inner;
  float* junction;
  int buf_elems;         // LDS-resident sweep: floats per interface buffer (BF16 planes: elements per plane)
  long long* clock;      // tracing (may be null): start/end clock per pair, then the workgroup
  int npairs;
  int stage;             // BF16-MFMA variant: the dynamic LDS holds a G_B stage after the interface planes
  int* claim;            // LDS-resident kernels: when set, workgroups claim positions of `order`
                         // (all npairs of them) from claim[0] and count exits in claim[1]; both are
                         // zero at launch and the last workgroup to exit clears them
};

// Level-by-level execution: one launch per step index from the right.
struct LevelItem {
  int pair;
  int rt;      // 16-row tile of V_k
};

struct LevelArgs {
  const PairDev* pairs;
  const int* ipool;
  const void* const* ppool;
  const LevelItem* items;  // items of this launch
  int level;               // step k = N - level of each item's pair
  unsigned ops;
  float* vbuf;             // two interface slots per pair
  const long* voff;        // per pair: offset of its slots in vbuf
  const long* vcap;        // per pair: elements per slot
  double* inner;
  float* junction;
  const float* one;        // V_N = [1]
};

hipError_t batch_set_lds(int bytes);
hipError_t level_set_lds(int level_bytes, int meet_bytes);
hipError_t launch_level(ttc_dtype dt, const LevelArgs& a, int nitems, size_t lds, hipStream_t s);
hipError_t launch_meet_level(ttc_dtype dt, const LevelArgs& a, int npairs, size_t lds, hipStream_t s);
hipError_t launch_batch(ttc_dtype dt, const BatchArgs& a, int grid, int threads, hipStream_t s);
// bytes: two interface buffers; stage_bytes: the BF16-MFMA variant's G_B stage (0 when off)
hipError_t batch_lds_set_lds(int bytes, int stage_bytes);
// Bytes of that stage: 128 rows of 40 BF16 (kStagePitch in sweep_lds16.hpp).
constexpr int kBatchStageBytes = 128 * 40 * 2;
// LDS-resident kernel variants: two FP32 interface buffers, one FP32 buffer
// updated in place, or (BF16 cores only) in place on BF16 MFMA with the
// interface as BF16 hi / lo planes.
enum { kBatchLdsTwo = 0, kBatchLdsInPlace = 1, kBatchLdsB16 = 2 };
hipError_t launch_batch_lds(ttc_dtype dt, const BatchArgs& a, int grid, int threads, int variant, hipStream_t s);

}  // namespace ttc
