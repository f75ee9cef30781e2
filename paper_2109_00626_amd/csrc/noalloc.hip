// Allocation-free inner product: tt_contract_inner with its workspace taken
// from a fixed device array of this library instead of the caller.  For
// callers that cannot allocate device memory (code under graph capture,
// tight serving loops, harnesses that forbid allocation).
//
// The array is a file-scope __device__ symbol: each device the library runs
// on holds its own copy, at its own address, until the process ends.  Host
// code never passes the symbol itself to a kernel (on the host it is only a
// stand-in); the device address comes from hipGetSymbolAddress, taken once
// per device with that device current and kept in a per-device table.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "ttc_internal.h"

namespace ttc {
ttc_status fail(ttc_status s, const std::string& msg);
}
using namespace ttc;

namespace {

static __device__ __align__(256) unsigned char scratch[TTC_NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch array.
ttc_status scratch_ptr(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(TTC_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return fail(TTC_ERR_UNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(TTC_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return TTC_OK;
}

}  // namespace

extern "C" {

ttc_status tt_contract_inner_noalloc(const ttc_tt* x, const ttc_tt* y, ttc_prec prec, double* d_out,
                                     void* stream) {
  size_t need = 0;
  ttc_status st = tt_contract_inner_query(x, y, prec, &need);
  if (st != TTC_OK) return st;
  if (need > (size_t)TTC_NOALLOC_SCRATCH_BYTES)
    return fail(TTC_ERR_WORKSPACE, "tt_contract_inner_noalloc: this pair needs " + std::to_string(need) +
                                       " bytes of workspace, the fixed scratch holds " +
                                       std::to_string((size_t)TTC_NOALLOC_SCRATCH_BYTES));
  void* ws = nullptr;
  st = scratch_ptr(&ws);
  if (st != TTC_OK) return st;
  return tt_contract_inner(x, y, prec, d_out, ws, (size_t)TTC_NOALLOC_SCRATCH_BYTES, stream);
}

}  // extern "C"
