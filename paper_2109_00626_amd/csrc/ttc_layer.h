// Internal interface of the TT-layer kernels (GEMM, permutations, loss).
#pragma once
#include <hip/hip_runtime.h>

#include "ttc_internal.h"

namespace ttc {

// Index map of a mixed-radix relayout: element (m, n) of an M x N matrix
// lives at
//   (m / (mr0 mr1)) ms2 + ((m / mr0) % mr1) ms1 + (m % mr0) ms0
//     + (n / nr0) ns1 + (n % nr0) ns0.
struct IdxMap {
  int mr0, mr1, nr0;
  long ms0, ms1, ms2, ns0, ns1;
};

// Output tile of the GEMM kernel (workgroup tile M x N).
enum GemmTile { GEMM_TILE_128x128 = 0, GEMM_TILE_32x128 = 1, GEMM_TILE_128x32 = 2, GEMM_TILE_128x64 = 3 };

// C (M x N, row-major, ldc) = alpha * A . B with
//   A(m, k) = a_kc ? A[m * lda + k] : A[k * lda + m]
//   B(k, n) = b_kc ? B[n * ldb + k] : B[k * ldb + n]
// splits > 1: K is cut into `splits` ranges whose partial products go to
// slab (splits x M x N) and are summed in order by a second kernel.
struct GemmArgs {
  int M, N, K;
  long lda, ldb, ldc;
  const float* A;
  const float* B;
  float* C;
  float alpha;
  int splits;
  float* slab;
  bool vec_a, vec_b;  // 16-byte vector loads allowed
  bool mapped;        // C element (m, n) goes to C[map(m, n)] (splits == 1)
  IdxMap map;
  GemmTile tile;
  // batch > 1 (splits == 1): `batch` independent products, the z-th on
  // A + z sa, B + z sb, C + z sc (a mapped store adds z sc to its map)
  int batch;
  long sa, sb, sc;
};

// dst[m * N + n] = src[map(m, n)] (the inverse of a mapped GEMM store).
struct GatherArgs {
  long M, N;
  IdxMap map;
  const float* src;
  float* dst;
};

struct PermArgs {
  int dir;            // 0: pair-mode order -> matrix, 1: matrix -> pair-mode order
  int d;
  int I[TTC_MAX_ORDER], J[TTC_MAX_ORDER];
  long pstride[TTC_MAX_ORDER];
  long cols;          // prod J
  long total;
  const float* src;
  float* dst;
};

// The same permutation by tiles staged in LDS.  A tile spans the digits
// that are contiguous in the pair-mode layout (i_{d-1}, j_{d-1}: Bp
// elements) and the t leading column digits j_0 .. j_{t-1}, contiguous in
// the matrix layout (Bm elements); both its read and its write are runs of
// consecutive addresses.  The other digits (outer) enumerate the tiles.
struct TilePermArgs {
  int dir;                        // as PermArgs
  int nout;                       // outer digits
  int orad[2 * TTC_MAX_ORDER];    // their radices (first varies fastest)
  long osP[2 * TTC_MAX_ORDER];    // their strides in the pair-mode layout
  long osM[2 * TTC_MAX_ORDER];    // and in the matrix layout
  int Bp, Jl;                     // I_{d-1} J_{d-1}, J_{d-1}
  long sMi, sMj;                  // matrix strides of i_{d-1}, j_{d-1}
  int t, Bm;                      // leading column digits, their product
  int jrad[TTC_MAX_ORDER];        // J_0 .. J_{t-1}
  long sPj[TTC_MAX_ORDER];        // their pair-mode strides
  long tiles;
  const float* src;
  float* dst;
  uint16_t* dst16;                // dir 0: BF16 destination instead of dst
  bool vec;                       // Bp, Bm multiples of 4: 16-byte global accesses
  FastDiv fgp, fgm, fjl;          // division by Bp / v, Bm / v and Jl (v = 4 if vec)
};

hipError_t launch_gemm(bool a_kc, bool b_kc, bool bf16, const GemmArgs& g, hipStream_t s);
// One FP32 product C = A . B on the GEMM kernel (layouts as in GemmArgs;
// map: the relayout store, else C row-major with ldc), split over K into
// `slab` (at most slab_elems floats) when the output has few tiles and a
// slab is given.  Defined with the TT layer's host code.
ttc_status gemm_f32(bool a_kc, const float* A, long lda, bool b_kc, const float* B, long ldb, float* C, long ldc,
                    int M, int N, int K, float* slab, size_t slab_elems, hipStream_t s, const IdxMap* map);
// `batch` such products (no split), the z-th on A + z sa, B + z sb and
// C + z sc (row-major with ldc, or through map when given).
ttc_status gemm_f32_batched(bool a_kc, const float* A, long lda, long sa, bool b_kc, const float* B, long ldb,
                            long sb, float* C, long ldc, long sc, int M, int N, int K, int batch, hipStream_t s,
                            const IdxMap* map);

// BF16 product C (M x N, FP32, ldc) = alpha * A . B^T for BF16 A (M x K) and
// B (N x K), both with k contiguous (lda, ldb multiples of 8, 16-byte
// aligned, K a multiple of 8); 256 x 256 tiles.  per_xcd: tiles per XCD
// when the tile count is a multiple of 8 (XCD-contiguous tile order), else 0.
struct Gemm16Args {
  int M, N, K;
  long lda, ldb, ldc;
  const uint16_t* A;
  const uint16_t* B;
  float* C;
  float alpha;
  int splits;
  float* slab;
  int per_xcd;
};
hipError_t gemm16_set_lds();
hipError_t launch_gemm16(const Gemm16Args& g, hipStream_t s);
// dst = bf16(src), n elements (n a multiple of 8; 16-byte aligned buffers)
hipError_t launch_cvt16(const float* src, uint16_t* dst, long n, hipStream_t s);
// dst (cols x rows) = bf16(src (rows x cols))^T
hipError_t launch_cvt16_t(const float* src, uint16_t* dst, long rows, long cols, hipStream_t s);
// both: dst = bf16(src), dst_t = bf16(src)^T, one read of src
hipError_t launch_cvt16_both(const float* src, uint16_t* dst, uint16_t* dst_t, long rows, long cols, hipStream_t s);
// Elements of the LDS tile of the tiled permutation (at most).
constexpr int kTilePermElems = 8192;
hipError_t launch_tile_permute(const TilePermArgs& p, hipStream_t s);
int gemm_bk(bool bf16);
// The tile for an M x N product (thin tiles for a side of at most 32 or 64)
// and its dimensions.
GemmTile gemm_tile(int M, int N);
void gemm_tile_dims(GemmTile t, int* tm, int* tn);
hipError_t launch_permute(const PermArgs& p, hipStream_t s);
hipError_t launch_gather(const GatherArgs& a, hipStream_t s);
// Core (R, I, J, R1) <-> its (J R) x (I R1) matrix Wp[(j, r), (i, r1)];
// dir 0: core -> Wp, dir 1: Wp -> core.
hipError_t launch_core_perm(const float* src, float* dst, int R, int I, int J, int R1, int dir, hipStream_t s);
int mse_blocks(long n);
hipError_t launch_mse(const float* y, const float* t, long n, float* dy, double* partials, double* out,
                      hipStream_t s);

}  // namespace ttc
