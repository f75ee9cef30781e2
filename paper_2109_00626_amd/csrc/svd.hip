// TT-SVD (Algorithm 1) on the GPU: the running unfolding of the tensor is
// split by a singular value decomposition N-1 times.
//
// Each SVD is a one-sided (Hestenes) Jacobi iteration on the rows of a
// p x L matrix A held in device memory: pairs of rows are rotated until every
// pair is orthogonal, and the same rotations are applied to a p x p matrix J
// that starts as the identity, so that A_final = J A_initial with J
// orthogonal and the rows of A_final mutually orthogonal; their norms are the
// singular values.  For an unfolding M (m x n):
//   m <= n: A = M.  Then M = J^T A_final: U = J^T (column c of U is row c of
//           J) and S V^T is A_final itself (row c = sigma_c v_c^T).
//   m >  n: A = M^T (a transposed copy).  Then M J^T = A_final^T has
//           orthogonal columns sigma_c u_c, so U[:, c] = A_final[c, :] /
//           sigma_c and S V^T = S J (row c = sigma_c J[c, :]).
// Either way only min(m, n) vectors are rotated, each of length max(m, n).
//
// The Jacobi kernel is one workgroup of 1024 threads: a sweep visits every
// pair once in the round-robin (circle) order, p-1 rounds of p/2 disjoint
// pairs (one row index fixed, the others rotating), one wave per pair at a
// time with FP64 dot products, a workgroup barrier between rounds.  Sweeps
// repeat until a whole sweep rotates nothing or the sweep limit is reached.
#include "ttc_device.hpp"
#include "ttc_internal.h"

namespace ttc {

namespace {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <typename T>
__device__ __forceinline__ double wide(T v) {
  return (double)v;
}

// Rows of length up to 64 x kJacobiChunk are held in registers per pair.
constexpr int kJacobiChunk = 8;

// The rotation (c, s) that zeroes the off-diagonal entry of the 2 x 2 Gram
// matrix [[al, ga], [ga, be]] (the smaller of the two equivalent angles).
__device__ __forceinline__ void jacobi_rotation(double al, double be, double ga, double* c, double* s) {
  const double zeta = (be - al) / (2.0 * ga);
  const double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
  *c = 1.0 / sqrt(1.0 + t * t);
  *s = *c * t;
}

}  // namespace

// out[c * m + r] = in[r * n + c] for an m x n row-major matrix, through
// 32 x 32 LDS tiles (both the reads and the writes run along rows).
template <typename T>
__global__ __launch_bounds__(256) void svd_transpose_kernel(const T* __restrict__ in, T* __restrict__ out, int m,
                                                            int n) {
  __shared__ T tile[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  const long r0 = (long)blockIdx.x * 32;  // row tiles on x (up to 2^31 - 1 tiles)
  const int c0 = blockIdx.y * 32;
#pragma unroll
  for (int q = 0; q < 32; q += 8) {
    const long r = r0 + ty + q;
    const int c = c0 + tx;
    if (r < m && c < n) tile[ty + q][tx] = in[r * n + c];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 32; q += 8) {
    const int c = c0 + ty + q;
    const long r = r0 + tx;
    if (r < m && c < n) out[(long)c * m + r] = tile[tx][ty + q];
  }
}

// One-sided Jacobi on the p rows (length L, row stride L) of A, rotations
// accumulated in J (p x p, set to the identity here).  sigma[i] = ||A[i, :]||
// at the end (FP64); info[0] = sweeps run, info[1] = 1 if the last sweep
// rotated nothing (converged).  A pair (i, j) is rotated when
// |a_i . a_j| > tol * ||a_i|| ||a_j||.
template <typename T>
__global__ __launch_bounds__(1024) void svd_jacobi_kernel(T* __restrict__ A, T* __restrict__ J, double* sigma,
                                                          int* info, int p, int L, int max_sweeps, double tol) {
  __shared__ int rotated;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (long e = threadIdx.x; e < (long)p * p; e += blockDim.x) {
    const int r = (int)(e / p), c = (int)(e - (long)r * p);
    J[e] = (r == c) ? T(1) : T(0);
  }
  const bool in_regs = L <= 64 * kJacobiChunk && p <= 64 * kJacobiChunk;
  const int pe = p + (p & 1);  // even count; index p (when p is odd) is a bye
  const int rounds = pe - 1, npairs = pe / 2;
  int sweep = 0, converged = 0;
  __syncthreads();
  while (sweep < max_sweeps) {
    if (threadIdx.x == 0) rotated = 0;
    __syncthreads();
    for (int rd = 0; rd < rounds; ++rd) {
      for (int k = wave; k < npairs; k += nw) {
        // circle method: slot 0 holds index 0, slot s >= 1 holds
        // 1 + (s - 1 + rd) mod (pe - 1); pair slots k and pe - 1 - k
        const int s1 = k, s2 = pe - 1 - k;
        const int i = s1 == 0 ? 0 : 1 + (s1 - 1 + rd) % (pe - 1);
        const int j = 1 + (s2 - 1 + rd) % (pe - 1);
        if (i >= p || j >= p) continue;
        T* ai = A + (long)i * L;
        T* aj = A + (long)j * L;
        T* ji = J + (long)i * p;
        T* jj = J + (long)j * p;
        if (in_regs) {
          // both rows of A and of J in registers: one load pass (all loads
          // in flight together) and one store pass per pair
          double xa[kJacobiChunk], ya[kJacobiChunk], xj[kJacobiChunk], yj[kJacobiChunk];
#pragma unroll
          for (int c = 0; c < kJacobiChunk; ++c) {
            const int t = lane + 64 * c;
            xa[c] = t < L ? wide(ai[t]) : 0.0;
            ya[c] = t < L ? wide(aj[t]) : 0.0;
            xj[c] = t < p ? wide(ji[t]) : 0.0;
            yj[c] = t < p ? wide(jj[t]) : 0.0;
          }
          double al = 0, be = 0, ga = 0;
#pragma unroll
          for (int c = 0; c < kJacobiChunk; ++c) {
            al += xa[c] * xa[c];
            be += ya[c] * ya[c];
            ga += xa[c] * ya[c];
          }
          al = __shfl(wave_sum(al), 0, 64);
          be = __shfl(wave_sum(be), 0, 64);
          ga = __shfl(wave_sum(ga), 0, 64);
          if (!(fabs(ga) > tol * sqrt(al * be))) continue;
          double c, s;
          jacobi_rotation(al, be, ga, &c, &s);
#pragma unroll
          for (int q = 0; q < kJacobiChunk; ++q) {
            const int t = lane + 64 * q;
            if (t < L) {
              ai[t] = (T)(c * xa[q] - s * ya[q]);
              aj[t] = (T)(s * xa[q] + c * ya[q]);
            }
            if (t < p) {
              ji[t] = (T)(c * xj[q] - s * yj[q]);
              jj[t] = (T)(s * xj[q] + c * yj[q]);
            }
          }
          if (lane == 0) rotated = 1;
          continue;
        }
        double al = 0, be = 0, ga = 0;
        for (int t = lane; t < L; t += 64) {
          const double x = wide(ai[t]), y = wide(aj[t]);
          al += x * x;
          be += y * y;
          ga += x * y;
        }
        // every lane takes lane 0's sums, so the whole wave makes the same
        // decision and applies the same rotation
        al = __shfl(wave_sum(al), 0, 64);
        be = __shfl(wave_sum(be), 0, 64);
        ga = __shfl(wave_sum(ga), 0, 64);
        if (!(fabs(ga) > tol * sqrt(al * be))) continue;
        double c, s;
        jacobi_rotation(al, be, ga, &c, &s);
        for (int q = lane; q < L; q += 64) {
          const double x = wide(ai[q]), y = wide(aj[q]);
          ai[q] = (T)(c * x - s * y);
          aj[q] = (T)(s * x + c * y);
        }
        for (int q = lane; q < p; q += 64) {
          const double x = wide(ji[q]), y = wide(jj[q]);
          ji[q] = (T)(c * x - s * y);
          jj[q] = (T)(s * x + c * y);
        }
        if (lane == 0) rotated = 1;
      }
      __syncthreads();
    }
    ++sweep;
    const int any = rotated;
    __syncthreads();
    if (!any) {
      converged = 1;
      break;
    }
  }
  for (int i = wave; i < p; i += nw) {
    const T* ai = A + (long)i * L;
    double s = 0;
    for (int t = lane; t < L; t += 64) {
      const double x = wide(ai[t]);
      s += x * x;
    }
    s = wave_sum(s);
    if (lane == 0) sigma[i] = sqrt(s);
  }
  if (threadIdx.x == 0) {
    info[0] = sweep;
    info[1] = converged;
  }
}

// One round of the same iteration spread over the GPU, for many vectors: a
// workgroup per pair of round `rd` (circle order as above), FP64 dot products
// reduced over the workgroup, the rotation applied to both rows of A and of
// J.  *rotated is set when a pair was rotated.  Consecutive rounds are
// consecutive launches (each round's pairs are disjoint, and the next round
// starts after this one ends).
template <typename T>
__global__ __launch_bounds__(256) void svd_round_kernel(T* __restrict__ A, T* __restrict__ J, int p, int L, int rd,
                                                        double tol, int* rotated) {
  __shared__ double red[3][4];
  const int pe = p + (p & 1);
  const int k = blockIdx.x;
  const int s1 = k, s2 = pe - 1 - k;
  const int i = s1 == 0 ? 0 : 1 + (s1 - 1 + rd) % (pe - 1);
  const int j = 1 + (s2 - 1 + rd) % (pe - 1);
  if (i >= p || j >= p) return;  // the bye: uniform over the workgroup
  T* ai = A + (long)i * L;
  T* aj = A + (long)j * L;
  double al = 0, be = 0, ga = 0;
  for (int t = threadIdx.x; t < L; t += blockDim.x) {
    const double x = wide(ai[t]), y = wide(aj[t]);
    al += x * x;
    be += y * y;
    ga += x * y;
  }
  al = wave_sum(al);
  be = wave_sum(be);
  ga = wave_sum(ga);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    red[0][wave] = al;
    red[1][wave] = be;
    red[2][wave] = ga;
  }
  __syncthreads();
  al = red[0][0] + red[0][1] + red[0][2] + red[0][3];
  be = red[1][0] + red[1][1] + red[1][2] + red[1][3];
  ga = red[2][0] + red[2][1] + red[2][2] + red[2][3];
  if (!(fabs(ga) > tol * sqrt(al * be))) return;  // uniform: every thread read the same sums
  double c, s;
  jacobi_rotation(al, be, ga, &c, &s);
  for (int q = threadIdx.x; q < L; q += blockDim.x) {
    const double x = wide(ai[q]), y = wide(aj[q]);
    ai[q] = (T)(c * x - s * y);
    aj[q] = (T)(s * x + c * y);
  }
  T* ji = J + (long)i * p;
  T* jj = J + (long)j * p;
  for (int q = threadIdx.x; q < p; q += blockDim.x) {
    const double x = wide(ji[q]), y = wide(jj[q]);
    ji[q] = (T)(c * x - s * y);
    jj[q] = (T)(s * x + c * y);
  }
  if (threadIdx.x == 0) *rotated = 1;
}

// J = identity (p x p) and sigma[i] = ||A[i, :]|| (FP64), one wave per row.
template <typename T>
__global__ __launch_bounds__(256) void svd_ident_kernel(T* __restrict__ J, int p) {
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < (long)p * p; e += (long)gridDim.x * blockDim.x) {
    const int r = (int)(e / p), c = (int)(e - (long)r * p);
    J[e] = (r == c) ? T(1) : T(0);
  }
}

template <typename T>
__global__ __launch_bounds__(256) void svd_norms_kernel(const T* __restrict__ A, double* sigma, int p, int L) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= p) return;
  const T* a = A + (long)row * L;
  double s = 0;
  for (int t = lane; t < L; t += 64) {
    const double x = wide(a[t]);
    s += x * x;
  }
  s = wave_sum(s);
  if (lane == 0) sigma[row] = sqrt(s);
}

// Core k and the next running matrix from the converged Jacobi state, for
// the r selected singular values sel[0..r) (in decreasing order):
//   G[row, c] (m x r): wide case J[sel_c, row]; tall case A[sel_c, row] / sigma_c;
//   C[c, col] (r x n): wide case A[sel_c, col]; tall case sigma_c J[sel_c, col].
template <typename T>
__global__ __launch_bounds__(256) void svd_split_kernel(const T* __restrict__ A, const T* __restrict__ J,
                                                        const double* __restrict__ sigma, const int* __restrict__ sel,
                                                        int tall, int m, int n, int p, int r, T* __restrict__ G,
                                                        T* __restrict__ C) {
  const long ng = (long)m * r, nc = (long)r * n;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < ng + nc; e += (long)gridDim.x * blockDim.x) {
    if (e < ng) {
      const int row = (int)(e / r), c = (int)(e - (long)row * r);
      const int q = sel[c];
      T v;
      if (!tall) {
        v = J[(long)q * p + row];
      } else {
        const double sg = sigma[q];
        v = sg > 0 ? (T)(wide(A[(long)q * m + row]) / sg) : T(0);
      }
      G[e] = v;
    } else {
      const long f = e - ng;
      const int c = (int)(f / n), col = (int)(f - (long)c * n);
      const int q = sel[c];
      C[f] = !tall ? A[(long)q * n + col] : (T)(sigma[q] * wide(J[(long)q * p + col]));
    }
  }
}

hipError_t launch_svd_transpose(ttc_dtype dt, const void* in, void* out, int m, int n, hipStream_t s) {
  const dim3 grid((unsigned)((m + 31) / 32), (unsigned)((n + 31) / 32));
  if (dt == TTC_F64)
    hipLaunchKernelGGL(svd_transpose_kernel<double>, grid, dim3(256), 0, s, (const double*)in, (double*)out, m, n);
  else
    hipLaunchKernelGGL(svd_transpose_kernel<float>, grid, dim3(256), 0, s, (const float*)in, (float*)out, m, n);
  return hipGetLastError();
}

hipError_t launch_svd_jacobi(ttc_dtype dt, void* A, void* J, double* sigma, int* info, int p, int L,
                             int max_sweeps, double tol, hipStream_t s) {
  if (dt == TTC_F64)
    hipLaunchKernelGGL(svd_jacobi_kernel<double>, dim3(1), dim3(1024), 0, s, (double*)A, (double*)J, sigma, info, p,
                       L, max_sweeps, tol);
  else
    hipLaunchKernelGGL(svd_jacobi_kernel<float>, dim3(1), dim3(1024), 0, s, (float*)A, (float*)J, sigma, info, p, L,
                       max_sweeps, tol);
  return hipGetLastError();
}

hipError_t launch_svd_round(ttc_dtype dt, void* A, void* J, int p, int L, int rd, double tol, int* rotated,
                            hipStream_t s) {
  const int npairs = (p + (p & 1)) / 2;
  if (dt == TTC_F64)
    hipLaunchKernelGGL(svd_round_kernel<double>, dim3(npairs), dim3(256), 0, s, (double*)A, (double*)J, p, L, rd,
                       tol, rotated);
  else
    hipLaunchKernelGGL(svd_round_kernel<float>, dim3(npairs), dim3(256), 0, s, (float*)A, (float*)J, p, L, rd, tol,
                       rotated);
  return hipGetLastError();
}

hipError_t launch_svd_ident(ttc_dtype dt, void* J, int p, hipStream_t s) {
  const int blocks = (int)std::min<long>(((long)p * p + 255) / 256, 4096);
  if (dt == TTC_F64)
    hipLaunchKernelGGL(svd_ident_kernel<double>, dim3(blocks), dim3(256), 0, s, (double*)J, p);
  else
    hipLaunchKernelGGL(svd_ident_kernel<float>, dim3(blocks), dim3(256), 0, s, (float*)J, p);
  return hipGetLastError();
}

hipError_t launch_svd_norms(ttc_dtype dt, const void* A, double* sigma, int p, int L, hipStream_t s) {
  const int blocks = (p + 3) / 4;
  if (dt == TTC_F64)
    hipLaunchKernelGGL(svd_norms_kernel<double>, dim3(blocks), dim3(256), 0, s, (const double*)A, sigma, p, L);
  else
    hipLaunchKernelGGL(svd_norms_kernel<float>, dim3(blocks), dim3(256), 0, s, (const float*)A, sigma, p, L);
  return hipGetLastError();
}

hipError_t launch_svd_split(ttc_dtype dt, const void* A, const void* J, const double* sigma, const int* sel,
                            int tall, int m, int n, int p, int r, void* G, void* C, hipStream_t s) {
  const long total = (long)m * r + (long)r * n;
  const int blocks = (int)std::min<long>((total + 255) / 256, 4096);
  if (dt == TTC_F64)
    hipLaunchKernelGGL(svd_split_kernel<double>, dim3(blocks), dim3(256), 0, s, (const double*)A, (const double*)J,
                       sigma, sel, tall, m, n, p, r, (double*)G, (double*)C);
  else
    hipLaunchKernelGGL(svd_split_kernel<float>, dim3(blocks), dim3(256), 0, s, (const float*)A, (const float*)J,
                       sigma, sel, tall, m, n, p, r, (float*)G, (float*)C);
  return hipGetLastError();
}

}  // namespace ttc

namespace ttc {

// C[r, c] = sum_k A[r, k] B[k, c] for row-major A (m x K) and B (K x n); one
// output per thread, FP64 sums.  The small products of TT-rounding (a core
// against a rank x rank factor).
template <typename T>
__global__ __launch_bounds__(256) void svd_small_gemm_kernel(const T* __restrict__ A, const T* __restrict__ B,
                                                             T* __restrict__ C, long m, int K, long n) {
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < m * n; e += (long)gridDim.x * blockDim.x) {
    const long r = e / n, c = e - r * n;
    const T* a = A + r * K;
    double acc = 0;
    for (int k = 0; k < K; ++k) acc += (double)a[k] * (double)B[(long)k * n + c];
    C[e] = (T)acc;
  }
}

// Right-orthogonalisation factors from a converged Jacobi state of an
// unfolding M (m x n, m = left bond): M = B Q with Q (r x n) orthonormal rows
// and B = U S (m x r), for the r = min(m, n) singular values in sel:
//   wide (A = M):    Q[c, :] = A[sel_c, :] / sigma_c;  B[:, c] = sigma_c J[sel_c, :]^T
//   tall (A = M^T):  Q[c, :] = J[sel_c, :];            B[:, c] = A[sel_c, :]^T
template <typename T>
__global__ __launch_bounds__(256) void svd_rsplit_kernel(const T* __restrict__ A, const T* __restrict__ J,
                                                         const double* __restrict__ sigma,
                                                         const int* __restrict__ sel, int tall, int m, int n, int p,
                                                         int r, T* __restrict__ Q, T* __restrict__ B) {
  const long nq = (long)r * n, nb = (long)m * r;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < nq + nb; e += (long)gridDim.x * blockDim.x) {
    if (e < nq) {
      const int c = (int)(e / n), col = (int)(e - (long)c * n);
      const int q = sel[c];
      if (!tall) {
        const double sg = sigma[q];
        Q[e] = sg > 0 ? (T)((double)A[(long)q * n + col] / sg) : T(0);
      } else {
        Q[e] = J[(long)q * p + col];
      }
    } else {
      const long f = e - nq;
      const int row = (int)(f / r), c = (int)(f - (long)row * r);
      const int q = sel[c];
      B[f] = !tall ? (T)(sigma[q] * (double)J[(long)q * p + row]) : A[(long)q * m + row];
    }
  }
}

hipError_t launch_svd_small_gemm(ttc_dtype dt, const void* A, const void* B, void* C, long m, int K, long n,
                                 hipStream_t s) {
  const long total = m * n;
  if (total <= 0) return hipSuccess;
  const int blocks = (int)std::min<long>((total + 255) / 256, 8192);
  if (dt == TTC_F64)
    hipLaunchKernelGGL(svd_small_gemm_kernel<double>, dim3(blocks), dim3(256), 0, s, (const double*)A,
                       (const double*)B, (double*)C, m, K, n);
  else
    hipLaunchKernelGGL(svd_small_gemm_kernel<float>, dim3(blocks), dim3(256), 0, s, (const float*)A,
                       (const float*)B, (float*)C, m, K, n);
  return hipGetLastError();
}

hipError_t launch_svd_rsplit(ttc_dtype dt, const void* A, const void* J, const double* sigma, const int* sel,
                             int tall, int m, int n, int p, int r, void* Q, void* B, hipStream_t s) {
  const long total = (long)r * n + (long)m * r;
  const int blocks = (int)std::min<long>((total + 255) / 256, 4096);
  if (dt == TTC_F64)
    hipLaunchKernelGGL(svd_rsplit_kernel<double>, dim3(blocks), dim3(256), 0, s, (const double*)A, (const double*)J,
                       sigma, sel, tall, m, n, p, r, (double*)Q, (double*)B);
  else
    hipLaunchKernelGGL(svd_rsplit_kernel<float>, dim3(blocks), dim3(256), 0, s, (const float*)A, (const float*)J,
                       sigma, sel, tall, m, n, p, r, (float*)Q, (float*)B);
  return hipGetLastError();
}

}  // namespace ttc
