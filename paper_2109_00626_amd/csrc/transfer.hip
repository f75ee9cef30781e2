// Two-sided transfer sweep: the junction of a contraction over a block of
// consecutive positions that need not touch either end of X or Y (eq. (8)
// applied once per contracted pair; Example 1's x_n^m at any n, m).  With
// a, b X's bonds before and after its block and g, d Y's, the block leaves
//   T[(a, g), (b, d)] = sum over the block's indices of X_block[a, .., b] Y_block[g, .., d],
// built one core pair at a time:
//   first pair:   E[(a, g), (b, d)] = sum_i Gx[a, i, b] Gy[g, i, d]
//   later pairs:  F[(a, g), g', i, b] = sum_a' E[(a, g), (a', g')] Gx[a', i, b]
//                 E'[(a, g), (b, d)] = sum_{g', i} F[(a, g), g', i, b] Gy[g', i, d]
// Each kernel writes one output entry per thread (grid-stride), reading the
// cores through the read-only cache; the sums run in the compute type (FP64
// for FP64 cores, FP32 otherwise) in a fixed order, so results are
// deterministic.
#include "ttc_device.hpp"
#include "ttc_internal.h"

namespace ttc {

// dab: E written as [d][(a, g)][b] (the layout the MFMA steps read)
// instead of [(a, g)][b][d].
template <typename Tin, typename Tc>
__global__ __launch_bounds__(256) void transfer_first_kernel(const Tin* __restrict__ gx, const Tin* __restrict__ gy,
                                                             int ka, int kg, int n, int kb, int kd, bool dab,
                                                             Tc* __restrict__ E) {
  const long total = (long)ka * kg * kb * kd;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    long r = e;
    int d, b;
    if (dab) {
      b = (int)(r % kb);
      r /= kb;
      const long rows = (long)ka * kg;
      d = (int)(r / rows);
      r -= (long)d * rows;
    } else {
      d = (int)(r % kd);
      r /= kd;
      b = (int)(r % kb);
      r /= kb;
    }
    const int g = (int)(r % kg);
    const int a = (int)(r / kg);
    const Tin* px = gx + (long)a * n * kb + b;
    const Tin* py = gy + (long)g * n * kd + d;
    Tc acc = 0;
    for (int i = 0; i < n; ++i) acc += cvt<Tc>(px[(long)i * kb]) * cvt<Tc>(py[(long)i * kd]);
    E[e] = acc;
  }
}

// F[(row), g', i, b] = sum_a' E[row, a' * kg1 + g'] Gx[a', i, b]; rows = ka * kg
// of E, whose columns are (a', g') with sizes (ka1, kg1).
template <typename Tin, typename Tc>
__global__ __launch_bounds__(256) void transfer_x_kernel(const Tc* __restrict__ E, const Tin* __restrict__ gx, long rows,
                                                         int ka1, int kg1, int n, int kb, Tc* __restrict__ F) {
  const long per_row = (long)kg1 * n * kb;
  const long total = rows * per_row;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const long row = e / per_row;
    long r = e - row * per_row;
    const int b = (int)(r % kb);
    r /= kb;
    const int i = (int)(r % n);
    const int g1 = (int)(r / n);
    const Tc* pe = E + row * ka1 * kg1 + g1;
    const Tin* px = gx + (long)i * kb + b;
    Tc acc = 0;
    for (int a1 = 0; a1 < ka1; ++a1) acc += pe[(long)a1 * kg1] * cvt<Tc>(px[(long)a1 * n * kb]);
    F[e] = acc;
  }
}

// E'[row, b * kd + d] = sum_{g', i} F[row, g', i, b] Gy[g', i, d].
template <typename Tin, typename Tc>
__global__ __launch_bounds__(256) void transfer_y_kernel(const Tc* __restrict__ F, const Tin* __restrict__ gy, long rows,
                                                         int kg1, int n, int kb, int kd, Tc* __restrict__ E) {
  const long per_row = (long)kb * kd;
  const long total = rows * per_row;
  const int red = kg1 * n;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const long row = e / per_row;
    const long r = e - row * per_row;
    const int b = (int)(r / kd), d = (int)(r - (long)b * kd);
    const Tc* pf = F + row * red * kb + b;
    const Tin* py = gy + d;
    Tc acc = 0;
    for (int gi = 0; gi < red; ++gi) acc += pf[(long)gi * kb] * cvt<Tc>(py[(long)gi * kd]);
    E[e] = acc;
  }
}

namespace {
int grid_for(long total) { return (int)std::min<long>((total + 255) / 256, 16384); }
}  // namespace

hipError_t launch_transfer_first(ttc_dtype dt, const void* gx, const void* gy, int ka, int kg, int n, int kb,
                                 int kd, bool dab, void* E, hipStream_t s) {
  const long total = (long)ka * kg * kb * kd;
  if (total <= 0) return hipSuccess;
  const int g = grid_for(total);
  switch (dt) {
    case TTC_F64:
      hipLaunchKernelGGL((transfer_first_kernel<double, double>), dim3(g), dim3(256), 0, s, (const double*)gx,
                         (const double*)gy, ka, kg, n, kb, kd, dab, (double*)E);
      break;
    case TTC_F32:
      hipLaunchKernelGGL((transfer_first_kernel<float, float>), dim3(g), dim3(256), 0, s, (const float*)gx,
                         (const float*)gy, ka, kg, n, kb, kd, dab, (float*)E);
      break;
    default:
      hipLaunchKernelGGL((transfer_first_kernel<bf16_t, float>), dim3(g), dim3(256), 0, s, (const bf16_t*)gx,
                         (const bf16_t*)gy, ka, kg, n, kb, kd, dab, (float*)E);
      break;
  }
  return hipGetLastError();
}

// BF16 core -> FP32 copy (exact), for the FP32 MFMA steps.
__global__ __launch_bounds__(256) void widen_kernel(const bf16_t* __restrict__ src, float* __restrict__ dst, long n) {
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
    dst[e] = cvt<float>(src[e]);
}

hipError_t launch_widen(const void* src, float* dst, long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(widen_kernel, dim3(grid_for(n)), dim3(256), 0, s, (const bf16_t*)src, dst, n);
  return hipGetLastError();
}

hipError_t launch_transfer_step(ttc_dtype dt, const void* E, const void* gx, const void* gy, long rows, int ka1,
                                int kg1, int n, int kb, int kd, void* F, void* Eout, hipStream_t s) {
  const long tf = rows * kg1 * n * kb, te = rows * kb * kd;
  if (tf <= 0 || te <= 0) return hipSuccess;
  switch (dt) {
    case TTC_F64:
      hipLaunchKernelGGL((transfer_x_kernel<double, double>), dim3(grid_for(tf)), dim3(256), 0, s, (const double*)E,
                         (const double*)gx, rows, ka1, kg1, n, kb, (double*)F);
      hipLaunchKernelGGL((transfer_y_kernel<double, double>), dim3(grid_for(te)), dim3(256), 0, s, (const double*)F,
                         (const double*)gy, rows, kg1, n, kb, kd, (double*)Eout);
      break;
    case TTC_F32:
      hipLaunchKernelGGL((transfer_x_kernel<float, float>), dim3(grid_for(tf)), dim3(256), 0, s, (const float*)E,
                         (const float*)gx, rows, ka1, kg1, n, kb, (float*)F);
      hipLaunchKernelGGL((transfer_y_kernel<float, float>), dim3(grid_for(te)), dim3(256), 0, s, (const float*)F,
                         (const float*)gy, rows, kg1, n, kb, kd, (float*)Eout);
      break;
    default:
      hipLaunchKernelGGL((transfer_x_kernel<bf16_t, float>), dim3(grid_for(tf)), dim3(256), 0, s, (const float*)E,
                         (const bf16_t*)gx, rows, ka1, kg1, n, kb, (float*)F);
      hipLaunchKernelGGL((transfer_y_kernel<bf16_t, float>), dim3(grid_for(te)), dim3(256), 0, s, (const float*)F,
                         (const bf16_t*)gy, rows, kg1, n, kb, kd, (float*)Eout);
      break;
  }
  return hipGetLastError();
}

}  // namespace ttc
