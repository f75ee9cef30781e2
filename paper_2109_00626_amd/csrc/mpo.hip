// TT-matrix (MPO) x TT-vector on cores:
//   C^(k)[(a,r), i, (a',r')] = sum_j W^(k)[a, i, j, a'] V^(k)[r, j, r'].
// For a fixed (a, i, r) the output row over (a', r') is contiguous, so one
// workgroup owns (core, a, i) and walks r: per r the product
//   D[r', a'] = sum_j V[r, j, r'] W[a, i, j, a']
// is a small GEMM (M = r', N = a', K = j) on 16x16x32 BF16 MFMA tiles with
// FP32 accumulation.  Both operands are staged in LDS with j contiguous, so
// every lane feeds the MFMA with one 16-byte read; every lane then writes 4
// consecutive r' of the output with one non-temporal 16-byte store.  The
// kernel is bound by the HBM write of the output (its entries outnumber the
// inputs' by orders of magnitude).
#include "ttc_device.hpp"
#include "ttc_internal.h"

namespace ttc {

#define MPO_WAVES 4

template <typename Tin, typename Tc>
__device__ __forceinline__ const MpoCore& find_core(const MpoArgs& a, int blk) {
  int c = 0;
  while (c + 1 < a.ncores && a.c[c + 1].blk_begin <= blk) ++c;
  return a.c[c];
}

// LDS row pitch (in bf16) for j: padded to a multiple of 32 plus 8 to spread banks.
__host__ __device__ __forceinline__ int mpo_pitch(int J) { return ((J + 31) / 32) * 32 + 8; }

__global__ __launch_bounds__(256) void mpo_bf16_kernel(MpoArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const MpoCore& c = find_core<bf16_t, float>(a, blockIdx.x);
  const int local = blockIdx.x - c.blk_begin;
  const int a_idx = local / c.I, i = local - a_idx * c.I;
  const int J = c.J, a1 = c.a1, r0 = c.r0, r1 = c.r1;
  const int pitch = mpo_pitch(J);
  const int Jp = ((J + 31) / 32) * 32;
  const int a1p = ((a1 + 15) / 16) * 16, r1p = ((r1 + 15) / 16) * 16;
  uint16_t* Wt = reinterpret_cast<uint16_t*>(smem);              // [a1p][pitch]
  uint16_t* Vt = Wt + a1p * pitch;                               // [MPO_WAVES][r1p][pitch]
  const uint16_t* Wsrc = reinterpret_cast<const uint16_t*>(c.w) + ((long)a_idx * c.I + i) * J * a1;
  const uint16_t* Vsrc = reinterpret_cast<const uint16_t*>(c.v);
  // stage W[a, i, :, :] transposed: Wt[a'][j]
  for (int e = threadIdx.x; e < a1p * Jp; e += blockDim.x) {
    const int ap = e / Jp, j = e - ap * Jp;
    Wt[ap * pitch + j] = (ap < a1 && j < J) ? Wsrc[(long)j * a1 + ap] : (uint16_t)0;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, g = lane >> 4;
  const long row_len = (long)a1 * r1;
  float* out_base = reinterpret_cast<float*>(c.out);
  const int tn = a1p / 16, tm = r1p / 16;
  for (int rb = 0; rb < r0; rb += MPO_WAVES) {
    __syncthreads();
    // stage V[r, :, :] transposed for the MPO_WAVES rows of this round
    for (int e = threadIdx.x; e < MPO_WAVES * r1p * Jp; e += blockDim.x) {
      const int w = e / (r1p * Jp);
      const int rem = e - w * r1p * Jp;
      const int j = rem / r1p, rp = rem - j * r1p;  // rp fastest: coalesced global reads
      const int r = rb + w;
      uint16_t v = 0;
      if (r < r0 && rp < r1 && j < J) v = Vsrc[((long)r * J + j) * r1 + rp];
      Vt[(w * r1p + rp) * pitch + j] = v;
    }
    __syncthreads();
    const int r = rb + wave;
    if (r >= r0) continue;
    float* orow = out_base + (((long)a_idx * r0 + r) * c.I + i) * row_len;
    const uint16_t* Vw = Vt + wave * r1p * pitch;
    for (int tt = 0; tt < tm * tn; ++tt) {
      const int m0 = (tt / tn) * 16, n0 = (tt % tn) * 16;
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
      for (int k0 = 0; k0 < Jp; k0 += 32) {
        const bf16x8 av = *reinterpret_cast<const bf16x8*>(Vw + (m0 + li) * pitch + k0 + 8 * g);
        const bf16x8 bv = *reinterpret_cast<const bf16x8*>(Wt + (n0 + li) * pitch + k0 + 8 * g);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc, 0, 0, 0);
      }
      const int ap = n0 + li;      // a'
      const int rp = m0 + 4 * g;   // first of 4 consecutive r'
      if (ap < a1) {
        float* q = orow + (long)ap * r1 + rp;
        if (rp + 3 < r1 && (r1 & 3) == 0) {
          __builtin_nontemporal_store(acc, reinterpret_cast<f32x4*>(q));
        } else {
          for (int v = 0; v < 4; ++v)
            if (rp + v < r1) q[v] = acc[v];
        }
      }
    }
  }
}

// Any dtype, plain FMA: one thread per output entry.
template <typename Tin, typename Tc>
__global__ __launch_bounds__(256) void mpo_generic_kernel(MpoArgs a) {
  const MpoCore& c = find_core<Tin, Tc>(a, blockIdx.x);
  const long per = (long)c.a0 * c.r0 * c.I * c.a1 * c.r1;
  const long e = (long)(blockIdx.x - c.blk_begin) * blockDim.x + threadIdx.x;
  if (e >= per) return;
  const int d1 = c.a1 * c.r1;
  const int col = (int)(e % d1);
  const long ri = e / d1;
  const int i = (int)(ri % c.I);
  const int row = (int)(ri / c.I);
  const int aa = row / c.r0, r = row - aa * c.r0;
  const int ap = col / c.r1, rp = col - ap * c.r1;
  const Tin* W = reinterpret_cast<const Tin*>(c.w) + (((long)aa * c.I + i) * c.J) * c.a1 + ap;
  const Tin* V = reinterpret_cast<const Tin*>(c.v) + (long)r * c.J * c.r1 + rp;
  Tc acc = 0;
  for (int j = 0; j < c.J; ++j) acc += cvt<Tc>(W[(long)j * c.a1]) * cvt<Tc>(V[(long)j * c.r1]);
  reinterpret_cast<Tc*>(c.out)[e] = acc;
}

size_t mpo_bf16_lds(const MpoArgs& a) {
  size_t mx = 0;
  for (int k = 0; k < a.ncores; ++k) {
    const MpoCore& c = a.c[k];
    const int pitch = mpo_pitch(c.J);
    const size_t b = ((size_t)((c.a1 + 15) / 16) * 16 + (size_t)MPO_WAVES * ((c.r1 + 15) / 16) * 16) * pitch * 2;
    if (b > mx) mx = b;
  }
  return mx;
}

hipError_t launch_mpo(ttc_dtype dt, bool bf16_mfma, const MpoArgs& in, hipStream_t s) {
  MpoArgs a = in;
  const size_t lds = bf16_mfma ? mpo_bf16_lds(a) : 0;
  const bool use_mfma = bf16_mfma && dt == TTC_BF16 && lds <= (size_t)lds_limit_bytes();
  int nblk = 0;
  for (int k = 0; k < a.ncores; ++k) {
    MpoCore& c = a.c[k];
    c.blk_begin = nblk;
    if (use_mfma) {
      nblk += c.a0 * c.I;
    } else {
      const long per = (long)c.a0 * c.r0 * c.I * c.a1 * c.r1;
      nblk += (int)((per + 255) / 256);
    }
  }
  a.nblk = nblk;
  if (nblk <= 0) return hipSuccess;
  if (use_mfma) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&mpo_bf16_kernel),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(mpo_bf16_kernel, dim3(nblk), dim3(64 * MPO_WAVES), lds, s, a);
    return hipGetLastError();
  }
  switch (dt) {
    case TTC_F64: hipLaunchKernelGGL((mpo_generic_kernel<double, double>), dim3(nblk), dim3(256), 0, s, a); break;
    case TTC_F32: hipLaunchKernelGGL((mpo_generic_kernel<float, float>), dim3(nblk), dim3(256), 0, s, a); break;
    default: hipLaunchKernelGGL((mpo_generic_kernel<bf16_t, float>), dim3(nblk), dim3(256), 0, s, a); break;
  }
  return hipGetLastError();
}

}  // namespace ttc
