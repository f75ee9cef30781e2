/*
 * ttc.h — C ABI of the MI355X (gfx950) library for tensor contraction
 * products computed directly on Tensor-Train (TT) cores.
 *
 * Method: Kisil, Calvi, Konstantinidis, Xu, Mandic, "Reducing Computational
 * Complexity of Tensor Contractions via Tensor-Train Networks"
 * (arXiv 2109.00626).  Section III contracts two tensors through their TT
 * cores (Algorithm 2); the first step of that contraction is the product of
 * the two first cores, K = A_x^T A_y.  This library generalises that step to
 * the interface sweep over a block of shared modes, and adds mode-n products
 * (Def. 5) and TT-matrix products on cores.
 *
 * Conventions (every call):
 *  - A TT of order N has mode sizes I[0..N-1] and ranks R[0..N] with
 *    R[0] = R[N] = 1 (Def. 7, eq. (9)).  Core k is one device buffer, a
 *    row-major (R[k], I[k], R[k+1]) array.  Modes are 0-based here; the
 *    paper counts from 1.
 *  - A TT-matrix (MPO) core k is a row-major (R[k], I[k], J[k], R[k+1]) array.
 *    Its dense matrix W[i, j] = prod_k W^(k)[:, i_k, j_k, :], with the row
 *    index i and column index j little-endian over (i_0..i_{N-1}) and
 *    (j_0..j_{N-1}), first index fastest (Def. 2, eq. (2) first line; Def. 3).
 *  - Dense multi-way outputs are ordinary row-major arrays indexed
 *    (i_0, ..., i_{n-1}); only flattened vectors (TT-matrix rows and
 *    columns, batch rows) use the little-endian index.
 *  - Pointers named d_* are device pointers; descriptor arrays (modes, ranks,
 *    core pointer lists) live in host memory and are read during the call
 *    only.  The caller owns every buffer.  The library never allocates on
 *    these calls: scratch memory comes from the caller as (d_ws, ws_bytes),
 *    sized by the matching *_query call.  Plans of the batched interface are
 *    the only library-owned objects.
 *  - `stream` is a hipStream_t passed as void* (0 = the null stream).  Calls
 *    are asynchronous on that stream and never synchronise the host, except
 *    tt_batch_plan_create.
 *  - Each call runs on the device current on the calling host thread; its
 *    buffers and stream must belong to that device, and a batched plan
 *    belongs to the device current when it was created.  Calls may come from
 *    several host threads at once; two calls that share a workspace or a
 *    plan must be ordered by the caller (one stream, or an event between).
 *  - Errors: every call validates all arguments on the host before any
 *    launch.  On error it returns a non-zero ttc_status, writes no output
 *    byte, and sets a thread-local message readable with ttc_last_error().
 *    No C++ exception crosses this interface.
 *  - Results are deterministic run to run (no floating-point atomics).
 */
#ifndef TTC_H
#define TTC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TTC_ABI_VERSION 2
#define TTC_MAX_ORDER 32 /* largest TT order accepted by single-pair calls */

typedef enum {
  TTC_OK = 0,
  TTC_ERR_NULL = 1,        /* a required pointer is NULL                         */
  TTC_ERR_SHAPE = 2,       /* mode sizes differ / do not match an operand        */
  TTC_ERR_RANK = 3,        /* boundary rank != 1, rank < 1, or rank mismatch     */
  TTC_ERR_MODE = 4,        /* mode index out of range or repeated                */
  TTC_ERR_DTYPE = 5,       /* dtype not supported or operands disagree           */
  TTC_ERR_UNSUPPORTED = 6, /* valid request this GPU path does not implement     */
  TTC_ERR_WORKSPACE = 7,   /* workspace smaller than the *_query size            */
  TTC_ERR_HIP = 8          /* a HIP runtime call or launch failed                */
} ttc_status;

typedef enum { TTC_F64 = 0, TTC_F32 = 1, TTC_BF16 = 2 } ttc_dtype;

/* Arithmetic precision.  AUTO: FP64 for FP64 inputs; FP32 interfaces with
 * FP32 accumulation for FP32 and BF16 inputs.  BF16: operands rounded to
 * BF16 (round to nearest even) on the matrix cores, FP32 accumulation.
 * Final scalars of inner products are always accumulated in FP64. */
typedef enum { TTC_PREC_AUTO = 0, TTC_PREC_F64 = 1, TTC_PREC_F32 = 2, TTC_PREC_BF16 = 3 } ttc_prec;

/* Output form of a partial contraction.
 *  JUNCTION: the matrix K joining X's free cores to Y's free cores (the K
 *            node of the paper's Fig. 3); free cores are not copied.
 *  NATURAL_TT: one TT over X's free modes then Y's (the mode order of
 *            eq. (8) and Algorithm 2's last step); the carried bond of K is
 *            lifted through the cores with merged index (own bond)*Q + q.
 *  DENSE:    the dense row-major result (small cases). */
typedef enum { TTC_JUNCTION = 0, TTC_NATURAL_TT = 1, TTC_DENSE = 2 } ttc_form;

/* Schedule of a TT-matrix x dense-batch product.  CORES: contract the batch
 * with one core at a time.  DENSE: rebuild the dense matrix from the cores,
 * then one matrix product.  AUTO picks the smaller FLOP count.
 * CORES_SAVED: CORES whose forward keeps every intermediate (one per core,
 * batch x prod(I_<k) x prod(J_>=k) x R_k elements) and the permuted cores in
 * the workspace, and whose backward reads them there instead of recomputing
 * the forward: the backward must get the same workspace, unmodified, with
 * the same cores, x, batch and prec as the forward that filled it (the
 * caller's contract, as for activations saved for a backward pass; it is
 * not checked).  Both directions query the backward's workspace size. */
typedef enum {
  TTC_SCHED_AUTO = 0,
  TTC_SCHED_CORES = 1,
  TTC_SCHED_DENSE = 2,
  TTC_SCHED_CORES_SAVED = 3
} ttc_sched;

/* TT tensor descriptor. */
typedef struct {
  int32_t order;          /* N >= 1                                         */
  const int32_t* modes;   /* host [N]: I[k] >= 1                            */
  const int32_t* ranks;   /* host [N+1]: ranks[0] = ranks[N] = 1            */
  ttc_dtype dtype;        /* element type of every core                     */
  void* const* cores;     /* host [N] of device pointers                    */
} ttc_tt;

/* TT-matrix (MPO) descriptor. */
typedef struct {
  int32_t order;
  const int32_t* rows;    /* host [N]: I[k], the output (row) modes          */
  const int32_t* cols;    /* host [N]: J[k], the input (column) modes        */
  const int32_t* ranks;   /* host [N+1]                                     */
  ttc_dtype dtype;
  void* const* cores;     /* host [N] of device pointers, (R, I, J, R')     */
} ttc_ttm;

/* ------------------------------------------------------------------------
 * Inner product <X, Y> = sum over all indices of X[i] Y[i]: the contraction
 * of two TTs along every mode (Fig. 1(b), all-mode contraction), computed by
 * interface sweeps.  Left to right, W_0 = [1] and
 *   W_k = sum_i G_x^(k)[:, i, :]^T W_{k-1} G_y^(k)[:, i, :]   (R_k x P_k);
 * the first step is the paper's K = A_x^T A_y (Section III, Example 1 and
 * Algorithm 2, step 4).  Right to left, V_N = [1] and
 *   V_{k-1} = sum_i G_x^(k)[:, i, :] V_k G_y^(k)[:, i, :]^T.
 * FP32 and BF16 pairs with every rank <= 128 keep the interfaces in LDS:
 * below order 4 one right-to-left sweep finished with the first cores in
 * FP64 (no workspace); from order 4 two such sweeps at once, V_c over cores
 * c..N-1 and W_c over the reversed prefix (c = N / 2; workspace: the two
 * R_c x P_c FP32 interfaces and rank-transposed copies of the prefix cores).
 * Otherwise the two sweeps meet at c in the chained-MFMA kernels.  Either
 * way z = sum W_c .* V_c, accumulated in FP64.  X and Y need equal order and
 * mode sizes; their ranks may differ.
 * x, y:   descriptors, same dtype.
 * prec:   AUTO, or the precision AUTO would pick, or BF16 for BF16 cores
 *         with every rank <= 128 (else TTC_ERR_UNSUPPORTED): the steps on
 *         BF16 MFMA, the interface carried as a BF16 hi / lo pair (about 16
 *         significant bits) with FP32 sums.
 * d_out:  device pointer to one double (written).
 * d_ws:   device scratch of at least the size tt_contract_inner_query
 *         returns (may be NULL when that size is 0).
 * ------------------------------------------------------------------------ */
ttc_status tt_contract_inner_query(const ttc_tt* x, const ttc_tt* y, ttc_prec prec,
                                   size_t* ws_bytes);
ttc_status tt_contract_inner(const ttc_tt* x, const ttc_tt* y, ttc_prec prec, double* d_out,
                             void* d_ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * tt_contract_inner without allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  Same arguments, kernels and result as
 * tt_contract_inner, but the workspace is a fixed array of
 * TTC_NOALLOC_SCRATCH_BYTES inside the library, one per GPU, held until the
 * process ends; the call itself allocates nothing.  A pair whose
 * tt_contract_inner_query size exceeds that returns TTC_ERR_WORKSPACE and
 * writes nothing.  Every call on one GPU shares that GPU's array: calls that
 * overlap in time on one GPU (different streams or host threads without an
 * ordering between them) race and may return wrong results.  No part of the
 * array needs to start at zero: each call writes every byte it reads.
 * ------------------------------------------------------------------------ */
#define TTC_NOALLOC_SCRATCH_BYTES (16u << 20)
ttc_status tt_contract_inner_noalloc(const ttc_tt* x, const ttc_tt* y, ttc_prec prec, double* d_out,
                                     void* stream);

/* ------------------------------------------------------------------------
 * Contraction of X and Y over a set of shared positions, each pair summed
 * as in eq. (8) (Def. 6).  The GPU path accepts a prefix {0..k-1}, a suffix
 * {k..N-1} or all positions, at equal positions and sizes in X and Y.
 * Prefix: K = W_k (R_k x P_k).  Suffix: K = V_k.  All: the scalar <X, Y>.
 *
 * modes / n_modes: host array of 0-based positions (any order, no repeats).
 * prec: as for tt_contract_inner (BF16: BF16 cores, every rank <= 128, the
 *       sweep on BF16 MFMA); the output forms are FP32 either way.
 * form: JUNCTION writes K (row-major, FP64 for FP64 inputs, FP32 otherwise)
 *       to out_junction; NATURAL_TT writes the cores of the natural-order TT
 *       into out_tt (shapes from the query; FP64 or FP32); DENSE writes the
 *       row-major dense tensor over (X free modes, Y free modes) to out_dense.
 *       When every position is contracted the scalar is written as one
 *       double to out_scalar whatever the form.
 * Natural-order construction (Q = columns of K, q its index):
 *   prefix: C_k[0, i, s*Q+q] = sum_r K[r,q] G_x^(k)[r,i,s];
 *           C_m[(s,q), i, (s',q')] = G_x^(m)[s,i,s'] delta(q,q') for m > k;
 *           then Y's cores k..N-1 unchanged.
 *   suffix: X's cores 0..k-2 unchanged; C_{k-1}[s,i,q] = sum_r G_x^(k-1)[s,i,r] K[r,q];
 *           Y's cores m < k-1: D_m[(p,q), j, (p',q')] = G_y^(m)[p,j,p'] delta(q,q');
 *           D_{k-1}[(p,q), j, 0] = G_y^(k-1)[p, j, q].
 * The query fills out_order, out_modes[<= 2N], out_ranks[<= 2N+1] (natural
 * TT or dense shape; junction: order 2 and K's shape in out_ranks[0..1]),
 * the output element count and the scratch size.
 * ------------------------------------------------------------------------ */
ttc_status tt_contract_modes_query(const ttc_tt* x, const ttc_tt* y, const int32_t* modes,
                                   int32_t n_modes, ttc_form form, ttc_prec prec,
                                   int32_t* out_order, int32_t* out_modes, int32_t* out_ranks,
                                   int64_t* out_elems, size_t* ws_bytes);
ttc_status tt_contract_modes(const ttc_tt* x, const ttc_tt* y, const int32_t* modes,
                             int32_t n_modes, ttc_form form, ttc_prec prec, void* out_junction,
                             const ttc_tt* out_tt, void* out_dense, double* out_scalar,
                             void* d_ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Mode-n products Y = X x_{n} A_n for every listed mode (Def. 5).  On a TT
 * only core n changes: G'[r, j, s] = sum_i A[j, i] G[r, i, s]; ranks are
 * unchanged and products on different modes commute.
 * count / modes: host list of distinct 0-based modes.
 * d_A[c]: device pointer to a row-major J[c] x I[modes[c]] matrix, x's dtype.
 * y: output descriptor (same order and ranks as x, mode modes[c] of size
 *    J[c]); only y->cores[modes[c]] are written, the other entries of
 *    y->cores are not touched (they may alias x's cores).
 * ------------------------------------------------------------------------ */
ttc_status tt_mode_n_product(const ttc_tt* x, int32_t count, const int32_t* modes,
                             const void* const* d_A, const int32_t* J, const ttc_tt* y,
                             void* stream);

/* ------------------------------------------------------------------------
 * TT-matrix times TT-vector on cores:
 *   C^(k)[(a,r), i, (a',r')] = sum_j W^(k)[a, i, j, a'] V^(k)[r, j, r'],
 * merged bond index a*R_v + r, output ranks the products of the input ranks.
 * m->cols must equal v->modes.  Output cores are FP32 for BF16/FP32 inputs
 * (FP32 accumulation; prec BF16 or AUTO uses the BF16 matrix cores for BF16
 * inputs) and FP64 for FP64 inputs.  The query returns the output ranks
 * (host array of order+1) and element count; `out` must have those shapes.
 * ------------------------------------------------------------------------ */
ttc_status ttm_apply_query(const ttc_ttm* m, const ttc_tt* v, int32_t* out_ranks,
                           int64_t* out_elems);
ttc_status ttm_apply(const ttc_ttm* m, const ttc_tt* v, ttc_prec prec, const ttc_tt* out,
                     void* stream);

/* ------------------------------------------------------------------------
 * TT-matrix times a dense batch (a TT layer): Y[b, :] = W X[b, :] for each
 * of `batch` rows; X is batch x prod(J) and Y is batch x prod(I), both
 * row-major FP32 with little-endian row vectors (Def. 3); the rows of the
 * batch are the stacking mode of Def. 4.  Cores are FP32.  prec AUTO/F32:
 * FP32 matrix cores; BF16: operands rounded to BF16, FP32 accumulation.
 * sched: see ttc_sched.  Backward: given dY, writes dX = dY W (skipped when
 * d_dx is NULL) and dW^(k) for every core into d_dcores[k] (FP32, the core's
 * shape; skipped when d_dcores is NULL).
 * ------------------------------------------------------------------------ */
ttc_status ttm_apply_dense_query(const ttc_ttm* m, int64_t batch, ttc_prec prec, ttc_sched sched,
                                 int32_t backward, size_t* ws_bytes);
ttc_status ttm_apply_dense(const ttc_ttm* m, const void* d_x, int64_t batch, void* d_y,
                           ttc_prec prec, ttc_sched sched, void* d_ws, size_t ws_bytes,
                           void* stream);
ttc_status ttm_apply_dense_bwd(const ttc_ttm* m, const void* d_x, const void* d_dy, int64_t batch,
                               void* d_dx, void* const* d_dcores, ttc_prec prec, ttc_sched sched,
                               void* d_ws, size_t ws_bytes, void* stream);

/* Mean squared error L = mean((y - t)^2) over n FP32 entries, accumulated
 * in FP64 into d_loss (one double), and dL/dy = 2 (y - t) / n into d_dy
 * (FP32, skipped when NULL).  Scratch: ttc_mse_loss_query bytes. */
ttc_status ttc_mse_loss_query(int64_t n, size_t* ws_bytes);
ttc_status ttc_mse_loss(const float* d_y, const float* d_t, int64_t n, double* d_loss, float* d_dy,
                        void* d_ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Gradient of z = <X, Y> with respect to every core, scaled by the upstream
 * gradient *d_gz (one device double):
 *   dz/dG_x^(k)[:, i, :] = W_k G_y^(k)[:, i, :] V_{k+1}^T,
 *   dz/dG_y^(k)[:, i, :] = W_k^T G_x^(k)[:, i, :] V_{k+1},
 * with W_k the left interface of core k and V_{k+1} the right one.
 * ckpt_stride > 0: a forward sweep keeps every ckpt_stride-th interface and
 * each segment between two kept ones is recomputed (memory for long trains).
 * ckpt_stride <= 0: FP32 and BF16 pairs with every rank <= 128 store every
 * interface from two LDS-resident sweeps (2 N max_k R_k P_k floats of
 * workspace); other pairs keep every ceil(sqrt(N))-th interface.
 * d_dx[k], d_dy[k]: device buffers shaped like the
 * cores, same dtype class (FP64 for FP64, FP32 otherwise); either list may
 * be NULL to skip that side.
 * ------------------------------------------------------------------------ */
ttc_status tt_contract_inner_bwd_query(const ttc_tt* x, const ttc_tt* y, int32_t ckpt_stride,
                                       size_t* ws_bytes);
ttc_status tt_contract_inner_bwd(const ttc_tt* x, const ttc_tt* y, const double* d_gz,
                                 void* const* d_dx, void* const* d_dy, int32_t ckpt_stride,
                                 void* d_ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Contraction of X's modes xmodes[l] with Y's modes ymodes[l], l < n_pairs
 * (eq. (8) once per pair, Def. 6; Example 1's X x_n^m Y is n_pairs = 1 at any
 * n, m).  X and Y may differ in order and in every mode outside the
 * contracted pairs.  The GPU path takes consecutive increasing blocks on
 * both sides (xmodes = a1..a2, ymodes = b1..b2) with equal sizes pairwise.
 * With a, b X's bonds before and after its block and g, d Y's, the blocks
 * leave the junction
 *   T[(a, g), (b, d)] = sum over the blocks' indices of X_block[a, .., b] Y_block[g, .., d],
 * a (R_a P_g) x (R_b P_d) matrix, row a * P_g + g, column b * P_d + d (a
 * prefix block's T holds W_k, a suffix block's V_k).  Forms:
 *   JUNCTION:   T to out_junction (FP64 for FP64 inputs, FP32 otherwise);
 *   NATURAL_TT: the cores of the result in eq. (8)'s mode order (X's free
 *               modes, then Y's) into out_tt (shapes from the query): X's
 *               cores left of the block copied, the first X core right of
 *               it absorbs T and carries q = g * P_d + d (Q = P_g P_d) through
 *               the rest, Y's cores left of its block carry q and the last of
 *               them contracts g, Y's cores right of its block copied;
 *               merged bonds are (own bond) * Q + q;
 *   DENSE:      the dense result (natural ranks <= 64).
 * Every position of both contracted: the scalar <X, Y> to out_scalar.  The
 * transfer runs one core pair at a time, T and its intermediate in the
 * workspace (each at most 2^28 elements).
 * tt_contract_pairs_query: out_order, out_modes (host, N + M - 2 n_pairs),
 * out_ranks (natural: order + 1; junction: the two sides of T), out_elems
 * and ws_bytes, any may be NULL.
 * ------------------------------------------------------------------------ */
ttc_status tt_contract_pairs_query(const ttc_tt* x, const ttc_tt* y, const int32_t* xmodes,
                                   const int32_t* ymodes, int32_t n_pairs, ttc_form form,
                                   int32_t* out_order, int32_t* out_modes, int32_t* out_ranks,
                                   int64_t* out_elems, size_t* ws_bytes);
ttc_status tt_contract_pairs(const ttc_tt* x, const ttc_tt* y, const int32_t* xmodes,
                             const int32_t* ymodes, int32_t n_pairs, ttc_form form,
                             void* out_junction, const ttc_tt* out_tt, void* out_dense,
                             double* out_scalar, void* d_ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * TT-SVD (Algorithm 1): the cores of a dense tensor X (row-major over
 * (i_1, ..., i_N), i_N fastest; FP64 or FP32, computed in that precision with
 * FP64 dot products).  delta = eps / sqrt(N-1) * ||X||_F; for k = 1..N-1 the
 * running unfolding (R_{k-1} I_k rows, row index r * I_k + i) is split by an
 * SVD, the kept rank R_k is the smallest whose discarded singular values have
 * norm <= delta (at most max_rank when max_rank > 0), core k is the first R_k
 * left singular vectors and the next running matrix S V^T of those.  eps = 0
 * keeps every nonzero singular value (the exact TT).
 *
 * tt_svd_query: rank_cap (host, N+1; may be NULL) gets the largest rank each
 *   bond can take; core k needs rank_cap[k] * dims[k] * rank_cap[k+1]
 *   elements.  ws_bytes: device workspace (three copies of X plus the SVD's
 *   p x p rotation matrix, p the smaller side of the widest unfolding, at
 *   most 4096: larger unfoldings return TTC_ERR_UNSUPPORTED).
 * tt_svd: ranks (host, N+1) receives the ranks; core k is written row-major
 *   (R_k, I_k, R_{k+1}) at the start of d_cores[k] (device, caller-owned,
 *   sized from rank_cap).  The ranks depend on the singular values, so the
 *   call synchronises `stream` once per split (N-1 times; once per Jacobi
 *   sweep for an unfolding with more than 32 rows and columns, whose rounds
 *   run as one launch each) and returns with the last copy queued.  X is
 *   not modified.
 * ------------------------------------------------------------------------ */
ttc_status tt_svd_query(int32_t order, const int32_t* dims, ttc_dtype dtype, int32_t max_rank,
                        int32_t* rank_cap, size_t* ws_bytes);
ttc_status tt_svd(const void* d_x, int32_t order, const int32_t* dims, ttc_dtype dtype, double eps,
                  int32_t max_rank, int32_t* ranks, void* const* d_cores, void* d_ws, size_t ws_bytes,
                  void* stream);

/* ------------------------------------------------------------------------
 * TT-rounding: the rule of Algorithm 1 applied to a TT given by its cores
 * (FP64 or FP32), without forming the dense tensor.  Right to left, each
 * core's unfolding (left bond x the rest) is split by the same Jacobi SVD
 * into orthonormal rows (the new core) and U S, which is multiplied into the
 * core on its left (exact zero singular values dropped); then left to right,
 * as in tt_svd, with delta = eps / sqrt(N-1) * ||X||_F and ranks at most
 * max_rank when max_rank > 0.  The result equals tt_svd of the dense tensor
 * up to the sign of each singular vector.  tt_round_query: rank_cap (host,
 * N+1; may be NULL) bounds each output bond, ws_bytes the workspace (N + 1
 * copies of the largest core, a p x p rotation matrix with p the smaller
 * side of the widest core unfolding, at most 4096).  tt_round: ranks (host,
 * N+1) receives the ranks, core k is written (R_k, I_k, R_{k+1}) at the start
 * of d_cores[k]; the input cores are not modified.  Synchronises `stream`
 * once per split (2N - 2 times), or once per Jacobi sweep as in tt_svd.
 * ------------------------------------------------------------------------ */
ttc_status tt_round_query(const ttc_tt* x, int32_t max_rank, int32_t* rank_cap, size_t* ws_bytes);
ttc_status tt_round(const ttc_tt* x, double eps, int32_t max_rank, int32_t* ranks, void* const* d_cores,
                    void* d_ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Batched execution: many independent pairs of uneven order, mode sizes and
 * ranks in one persistent launch, replayed from a HIP graph.  For each pair
 * p the right-to-left sweep gives both results:
 *   TTC_OP_INNER:   d_inner[p] = <X_p, Y_p> (FP64);
 *   TTC_OP_SUFFIX2: the junction K = V_{N-2} of the contraction over the last
 *                   two positions, row-major FP32 at d_junction +
 *                   junction_offset[p] elements (offsets from
 *                   tt_batch_plan_info).
 * Pairs need order >= 2 (SUFFIX2: >= 3) and order <= 32; X and Y of a pair
 * share dtype (FP32 or BF16) and mode sizes.  prec: AUTO lets the tuner pick
 * among every schedule; F32 keeps the steps on FP32 MFMA (BF16 cores are
 * widened); BF16 (BF16 cores only, else TTC_ERR_UNSUPPORTED) runs every step
 * on BF16 MFMA with FP32 sums (mode 4 below).  The plan copies every
 * descriptor (shapes and core pointers) when it is created; the core buffers
 * must stay alive and unchanged in place until the plan is destroyed.
 * tt_batch_plan_create synchronises the device once (descriptor upload and
 * tile selection).  The LDS-resident schedules (modes 2 and 3 below) hand
 * pairs to workgroups through a work counter owned by the plan, so runs of
 * one plan (tt_batch_run, tt_batch_run_traced) must not overlap in time:
 * issue them on one stream, or order them with events.  Different plans are
 * independent.
 * ------------------------------------------------------------------------ */
typedef struct {
  ttc_tt x;
  ttc_tt y;
} ttc_pair;

typedef struct ttc_plan ttc_plan;

#define TTC_OP_INNER 1u
#define TTC_OP_SUFFIX2 2u

ttc_status tt_batch_plan_create(const ttc_pair* pairs, int32_t n, uint32_t ops, ttc_prec prec,
                                ttc_plan** plan);
/* The plan's host-side bookkeeping without creating a plan (no device
 * call): the same validation as tt_batch_plan_create; junction_offsets (n+1
 * int64: prefix sums of R_{N-2} P_{N-2} per pair with SUFFIX2, else zeros),
 * the algorithmic FLOPs (the cheaper contraction order of every
 * right-to-left step, the first cores' product and the final sum) and bytes
 * (every core read once, the FP64 scalar and the FP32 junction written once)
 * of one run, each pair's modelled cost (shader cycles of one workgroup) and
 * claim_order (n int32: pairs by decreasing cost, ties in index order, the
 * order in which the LDS-resident schedules' workgroups claim them).  Every
 * output is a host array and may be NULL. */
ttc_status tt_batch_plan_query(const ttc_pair* pairs, int32_t n, uint32_t ops, int64_t* junction_offsets,
                               double* flops, double* bytes, double* cost, int32_t* claim_order);
/* junction_offsets: host array of n+1 int64 (may be NULL); flops / bytes:
 * algorithmic FLOPs and bytes of one run (may be NULL). */
ttc_status tt_batch_plan_info(const ttc_plan* plan, int64_t* junction_offsets, double* flops,
                              double* bytes);
/* The schedule the plan's tuner selected (host ints; any may be NULL):
 * mode 0 = persistent kernel with chained-MFMA steps, 1 = one launch per
 * sweep level, 2 = persistent kernel with LDS-resident interfaces, 3 = the
 * same with one interface buffer per workgroup updated in place, 4 (BF16
 * cores only) = mode 3 on BF16 MFMA with the interface held as a BF16 hi /
 * lo pair (16 significant bits);
 * threads = workgroup size; wg_per_cu = workgroups per compute unit. */
ttc_status tt_batch_plan_config(const ttc_plan* plan, int32_t* mode, int32_t* threads, int32_t* wg_per_cu);
/* One run of the plan: the selected schedule's launch(es), captured once per
 * (d_inner, d_junction) pair into a HIP graph on the plan's own stream and
 * replayed on `stream` (any stream, the null stream included).  The plan
 * keeps the graphs of the last four output-pointer pairs; an older one is
 * destroyed only after its last replay has finished (an event recorded
 * after every replay). */
ttc_status tt_batch_run(ttc_plan* plan, double* d_inner, float* d_junction, void* stream);
/* The same pairs as one single-pair launch sequence each (the plain loop
 * that the batched launch replaces); same outputs. */
ttc_status tt_batch_run_plain(ttc_plan* plan, double* d_inner, float* d_junction, void* stream);
/* tt_batch_run with tracing: the same outputs, plus GPU clock readings
 * (s_memtime, shader cycles; comparable within one workgroup) in d_clock, a
 * device int64 array of 35 n entries: for pair p, d_clock[2p] and
 * d_clock[2p+1] are when its workgroup started and finished it,
 * d_clock[2n + p] is that workgroup, and d_clock[3n + 32p + j] the clock
 * after sweep step j (j = 0 .. N-2, right to left) and, at j = N-1, after
 * the final product.  Launched directly (not from the plan's graph); for
 * load-balance and per-step cost analysis. */
ttc_status tt_batch_run_traced(ttc_plan* plan, double* d_inner, float* d_junction, int64_t* d_clock,
                               void* stream);
void tt_batch_plan_destroy(ttc_plan* plan);

/* ------------------------------------------------------------------------ */
const char* ttc_last_error(void); /* thread-local; "" when none            */
const char* ttc_version(void);
int32_t ttc_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* TTC_H */
