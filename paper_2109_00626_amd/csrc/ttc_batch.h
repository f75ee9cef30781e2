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
};

hipError_t batch_set_lds(int bytes);
hipError_t launch_batch(ttc_dtype dt, const BatchArgs& a, int grid, int threads, hipStream_t s);

}  // namespace ttc
