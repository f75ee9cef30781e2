// Mode-n products on TT cores (Def. 5): X x_n A changes only core n,
//   G'[r, j, s] = sum_i A[j, i] G[r, i, s].
// One launch covers every listed mode; each thread writes one output entry.
#include "ttc_device.hpp"
#include "ttc_internal.h"

namespace ttc {

template <typename Tin, typename Tc>
__global__ __launch_bounds__(256) void mode_n_kernel(ModeNArgs a) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= a.total) return;
  int c = 0;
  while (c + 1 < a.count && a.e[c + 1].first <= e) ++c;
  const ModeNEntry& m = a.e[c];
  const long l = e - m.first;
  const int s = (int)(l % m.r1);
  const long rj = l / m.r1;
  const int j = (int)(rj % m.J);
  const int r = (int)(rj / m.J);
  const Tin* G = reinterpret_cast<const Tin*>(m.src) + (long)r * m.I * m.r1 + s;
  const Tin* A = reinterpret_cast<const Tin*>(m.A) + (long)j * m.I;
  Tc acc = 0;
  for (int i = 0; i < m.I; ++i) acc += cvt<Tc>(A[i]) * cvt<Tc>(G[(long)i * m.r1]);
  store_as(reinterpret_cast<Tin*>(m.dst) + l, acc);
}

hipError_t launch_mode_n(ttc_dtype dt, const ModeNArgs& a, hipStream_t s) {
  if (a.total <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)((a.total + 255) / 256);
  switch (dt) {
    case TTC_F64: hipLaunchKernelGGL((mode_n_kernel<double, double>), dim3(blocks), dim3(256), 0, s, a); break;
    case TTC_F32: hipLaunchKernelGGL((mode_n_kernel<float, float>), dim3(blocks), dim3(256), 0, s, a); break;
    default: hipLaunchKernelGGL((mode_n_kernel<bf16_t, float>), dim3(blocks), dim3(256), 0, s, a); break;
  }
  return hipGetLastError();
}

}  // namespace ttc
