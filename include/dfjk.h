/*
 * dfjk.h -- C ABI of the MI355X (gfx950) density-fitting Coulomb/exchange build.
 *
 * The library computes, for a whitened three-index tensor B[P][mu][nu]
 * (naux x nao x nao, symmetric in mu, nu), occupied orbitals C[nu][i]
 * (nao x nocc) and the density D = occ * C C^T:
 *
 *   rho_P      = sum_{mu,nu} B[P][mu][nu] D[mu][nu]          (Sec. 2.1, Eq. 3)
 *   J[mu][nu]  = sum_P rho_P B[P][mu][nu]                     (Eq. 4)
 *   X[P][mu][i]= sum_nu B[P][mu][nu] C[nu][i]                 (Eq. 5; the paper's W)
 *   K[mu][nu]  = occ * sum_{P,i} X[P][mu][i] X[P][nu][i]      (Eq. 6)
 *   E_J = 1/2 sum_P rho_P^2,   E_x = -1/4 sum_{mu,nu} D K
 *
 * K is formed per block of `pblk` consecutive aux indices (Eqs. df-k-blk-1/2
 * of Sec. 3.3).  Its two products run either in native FP64 (slices = 0) or
 * as FP64 emulated by s = 1..8 INT8 slices (Sec. 3.2: s = ceil((m + 1) / 8)
 * splits for m mantissa bits):
 *   - every operand row r (over the contraction index) gets the power-of-two
 *     exponent e_r of its largest magnitude; trunc(a * 2^(62 - e_r)) is split
 *     into balanced base-256 digits d_1..d_8 (d_1 most significant), of which
 *     a level-s slicing keeps d_1..d_s;
 *   - the s(s+1)/2 digit products with a + b <= s + 1 are accumulated exactly
 *     in int32, one accumulator per anti-diagonal g = a + b;
 *   - FP64 recombination: Z = sum_{g = s+1 .. 2} ldexp(S_g, e_r + f_c + 4 - 8g),
 *     smallest weight first.
 * In df_build_jk, J and rho are FP64 at every precision (the paper keeps J in
 * FP64, Sec. 3).  The sliced mode (df_prepare_b / df_build_jk_sliced) also
 * forms rho and J from the INT8 digits of B, with FP64 recombination.
 *
 * Conventions for every entry point:
 *   - Array arguments are DEVICE pointers to caller-owned memory (allocated by
 *     the caller, e.g. through PyTorch).  The library never frees or keeps them
 *     after the call returns.  Arrays are row-major and C-contiguous; double
 *     arrays must be 8-byte aligned, int8 arrays 16-byte aligned.
 *   - Work is enqueued asynchronously on the context's HIP stream; outputs are
 *     valid after that stream is synchronised.
 *   - Return value: DF_OK (0) or a negative DF_E* code.  Argument errors are
 *     reported synchronously and enqueue nothing; df_last_error() gives text.
 *     Data errors found on the device (a NaN or Inf in a sliced operand) set
 *     a status word that df_get_status() reads (it synchronises the stream).
 *   - One context per stream; a context is not thread-safe.
 *   - HIP graphs: df_density, df_build_x, df_build_jk and df_build_jk_batched
 *     enqueue kernels (and, batched, event records and waits that fork and
 *     join its worker streams) and nothing else: no memset, allocation or
 *     synchronisation.  They may be captured in a graph on the context stream;
 *     the batched build once a first eager call has created its worker
 *     streams.  Replays read and write the buffers given at capture.
 */
#ifndef DFJK_H
#define DFJK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum df_status {
  DF_OK = 0,
  DF_EINVAL = -1,          /* bad shape, pointer, slice count or layout          */
  DF_EWORKSPACE = -2,      /* workspace missing or smaller than df_workspace_size */
  DF_EHIP = -3,            /* a HIP runtime call failed                          */
  DF_ENONFINITE = -4,      /* NaN/Inf met while slicing (device status)          */
  DF_EOVERFLOW_GUARD = -5, /* s * pblk * nocc * 2^14 >= 2^31: int32 sums unsafe  */
  DF_ENOTSPD = -6          /* non-positive pivot in the metric Cholesky (device)  */
};

/* Storage of the three-index tensor B (every B_P is symmetric):
 *   DF_DENSE  [naux][nao][nao], both triangles.
 *   DF_PACKED [naux][nao (nao + 1) / 2], the lower triangle of each B_P by
 *             rows: element (mu, nu), mu >= nu, at mu (mu + 1) / 2 + nu (the
 *             stored form of Sec. 3.3; half the bytes).  nao <= 16383.  Taken
 *             by df_b_exponents, df_build_x, df_build_jk, df_build_jk_noalloc,
 *             df_prepare_b, df_spot_check and df_debug_build_i32; results are
 *             bit-identical to the same build on the dense tensor, except rho
 *             (and so J and E_J), which may differ in FP64 rounding order.
 *             Screening, the autotuner and the batched build take DF_DENSE. */
enum df_layout {
  DF_DENSE = 0,
  DF_PACKED = 1
};

typedef struct df_ctx df_ctx;

/* Create a context bound to `hip_stream` (a hipStream_t; NULL = null stream).
 * Precision starts at 0 (native FP64), the aux block size at 64. */
int df_create(df_ctx** ctx, void* hip_stream);

/* Destroy a context (does not touch caller memory).  NULL is ignored. */
void df_destroy(df_ctx* ctx);

/* Slice count used by df_build_jk / df_build_x: 0 = native FP64 MFMA,
 * 1..8 = INT8 slices (Table 1 of the paper uses 3..6).  DF_EINVAL otherwise. */
int df_set_precision(df_ctx* ctx, int slices);
int df_get_precision(const df_ctx* ctx);

/* Per-aux-block slice counts for df_build_jk (the learned controller's
 * decisions; per-block precision extends the per-iteration rule of Sec. 3.2,
 * Table 1, in the direction of Sec. 5): host_s[b] in 0..8 for each of the
 * nblocks = ceil(naux / pblk) aux blocks, 0 = native FP64 for that block.
 * X_b and K_b of block b are then formed at host_s[b]; each block gets its
 * own K partial (the K group count becomes nblocks), summed in ascending
 * block order; err_bound uses each block's own factors.  Set it before
 * df_workspace_size.  The counts are copied (the call synchronises the
 * context stream and may allocate a small device array owned by the
 * context); host_s == NULL returns to the context precision for all blocks.
 * df_build_x and df_build_jk_sliced do not take per-block counts
 * (df_build_jk_sliced returns DF_EINVAL while they are set); df_build_jk
 * returns DF_EINVAL when nblocks does not match its shape. */
int df_set_block_precision(df_ctx* ctx, const int32_t* host_s, int64_t nblocks);

/* Aux block size of the blocked K (Eqs. df-k-blk-1/2): 1..1024 (default 64). */
int df_set_pblk(df_ctx* ctx, int pblk);

/* Number of contiguous groups of aux blocks whose exchange partial sums are
 * formed independently and then added in ascending group order (0 = let the
 * library choose from the problem shape; the value used by the last build is
 * returned by df_get_k_groups).  Within a group the blocks are added in
 * ascending order, so the emulated K is deterministic for a given value. */
int df_set_k_groups(df_ctx* ctx, int groups);
int df_get_k_groups(const df_ctx* ctx);

/* Digit-pair scheme of the emulated products: extra = 0 forms the pairs
 * a + b <= s + 1 (s(s+1)/2 INT8 products; Sec. 3.2, Eq. 8), extra = 1 also
 * the anti-diagonal a + b = s + 2 (s - 1 more products, a, b <= s): the
 * dropped-pair error shrinks, so the stated bound is tighter at s <= 7 for the
 * same slice count (an alternative scheme along the outlook of Sec. 5 on
 * choosing slice counts; at s = 1 there is nothing to add).  Applies to
 * df_build_jk, df_build_x and df_debug_build_i32 (which then exports s + 1
 * anti-diagonals); df_build_jk_sliced returns DF_EINVAL while extra = 1.
 * DF_EINVAL outside 0..1. */
int df_set_extra_pairs(df_ctx* ctx, int extra);

/* Depth of the nu chunk that one step of the INT8 X product stages in LDS:
 * 1 = 64 (two LDS stages, the default), 2 = 128 (one stage; used only where
 * slices <= 5 and nao is a multiple of 128, else 64), 0 = the autotuned choice
 * of df_autotune for the shape, else the default.  Results are identical at
 * every depth (the int32 sums are exact).  DF_EINVAL outside 0..2. */
int df_set_x_ksub(df_ctx* ctx, int ksub);

/* Bytes of device workspace needed by df_build_jk / df_build_x for this shape
 * at any precision.  The caller allocates it and hands it over with
 * df_set_workspace (the library only borrows it until the next call). */
int df_workspace_size(df_ctx* ctx, int64_t naux, int64_t nao, int64_t nocc, int layout,
                      size_t* bytes);
int df_set_workspace(df_ctx* ctx, void* dev_ptr, size_t bytes);

/* Row exponents of B over nu: b_exp[P*nao + mu] = e with
 * 2^(e-1) <= max_nu |B[P][mu][nu]| < 2^e (0 for an all-zero row).
 * B does not change across SCF iterations, so callers compute this once and
 * pass it to every df_build_jk / df_build_x call.  Non-finite B sets the
 * DF_ENONFINITE device status. */
int df_b_exponents(df_ctx* ctx, const double* B, int layout, int64_t naux, int64_t nao,
                   int32_t* b_exp);

/* Slice the rows of A (rows x cols, leading dimension lda >= cols) at level
 * `slices` (1..8): digits[a][r][c] (int8, a = 0 is the most significant
 * digit d_1) and row_exp[r] as defined above.  Sec. 3.2 / Sec. 2.3, Eq. 8. */
int df_slice(df_ctx* ctx, const double* A, int64_t rows, int64_t cols, int64_t lda,
             int slices, int8_t* digits, int32_t* row_exp);

/* Eq. (5) alone at the context precision: X[P][mu][i] (naux x nao x nocc).
 * b_exp may be NULL (it is then computed into the workspace). */
int df_build_x(df_ctx* ctx, const double* B, int layout, int64_t naux, int64_t nao,
               const int32_t* b_exp, const double* C, int64_t nocc, double* X);

/* The whole build at the context precision (Eqs. 3-6).
 *   B       [naux][nao][nao] (DF_DENSE) or [naux][nao (nao + 1) / 2] (DF_PACKED),
 *           symmetric in the last two indices
 *   b_exp   [naux*nao] from df_b_exponents, or NULL
 *   C       [nao][nocc];  occ the occupation factor (2 for closed shells)
 *   D       [nao][nao], the density occ * C C^T used for rho (Eq. 3); symmetric, like
 *           each B_P: at 1..7 slices with nao a multiple of 64, rho sums the 64 x 64
 *           blocks on and below the diagonal of B_P o D, those below counted twice
 *           (the same sum in another rounding order)
 *   J, K    [nao][nao] outputs (both written in full, symmetric)
 *   energies[2] output: E_J, E_x
 *   err_bound[1] output: an upper bound on max |K - K_exact| (absolute) that
 *           covers the slicing, the dropped digit pairs and FP64 rounding of
 *           the emulated products (s >= 1), or the FP64 dot-product bound (s = 0).
 * Requires a workspace of df_workspace_size bytes. */
int df_build_jk(df_ctx* ctx, const double* B, int layout, int64_t naux, int64_t nao,
                const int32_t* b_exp, const double* C, int64_t nocc, double occ,
                const double* D, double* J, double* K, double* energies, double* err_bound);

/* df_build_jk without a caller workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Arguments, results and errors are those of
 * df_build_jk; the workspace is a static device array of 64 MiB that every
 * device holds from the load of the library until the process ends (its
 * address is looked up by df_create).  Shapes whose df_workspace_size exceeds
 * 64 MiB return DF_EWORKSPACE (about nao <= 160 with naux = 4 nao and nocc =
 * nao / 8; nao 96, naux 384, nocc 16 needs 15 MiB); the call
 * allocates nothing and does not touch the context's own workspace.  All
 * calls on one device share that array, which keeps the last call's contents:
 * calls that overlap in time on one device (several streams or contexts)
 * race; calls ordered on one stream do not. */
int df_build_jk_noalloc(df_ctx* ctx, const double* B, int layout, int64_t naux, int64_t nao,
                        const int32_t* b_exp, const double* C, int64_t nocc, double occ,
                        const double* D, double* J, double* K, double* energies,
                        double* err_bound);

/* Sliced mode, step 1 (once per B; Sec. 3.2 splitting applied to B itself):
 * b_exp[P*nao + mu] as in df_b_exponents and the first `planes` (1..8) digit
 * planes of every row (P, mu) of B over nu:
 *   b_dig[a][P*nao + mu][c], a = 0..planes-1 (a = 0 is d_1), c < ldk,
 *   ldk = nao rounded up to a multiple of 64, columns c >= nao zero.
 * df_prepare_b_size gives the byte count of b_dig (planes * naux * nao * ldk);
 * b_dig must be 16-byte aligned.  Any prefix of the planes serves every level
 * s <= planes.  Non-finite B sets the DF_ENONFINITE device status.  No
 * workspace. */
int df_prepare_b_size(int64_t naux, int64_t nao, int planes, size_t* bytes);
int df_prepare_b(df_ctx* ctx, const double* B, int layout, int64_t naux, int64_t nao, int planes,
                 int32_t* b_exp, int8_t* b_dig);

/* Sliced mode, step 2: the build of df_build_jk (Eqs. 3-6) with every product
 * over B taken from its digit planes at the context precision s
 * (1 <= s <= planes; DF_EINVAL otherwise):
 *   X = B C and K exactly as df_build_jk at level s (bitwise the same);
 *   rho_P = sum over mu (ascending) of the emulated row dot
 *     B[P][mu][:] . D[mu][:] (rows of D sliced over nu, s pairs rule);
 *   J[mu][nu] (nu <= mu, mirrored) = emulated sum_P w[P][mu] B~[P][mu][nu]
 *     with w[P][mu] = rho_P 2^b_exp[P*nao+mu], sliced over P for each mu, and
 *     B~ = B / 2^b_exp (whose digits are b_dig).
 * Arguments as df_build_jk, except b_dig / planes / b_exp from df_prepare_b
 * (B itself is not read) and err_bound[2]: err_bound[0] bounds max |K - K_exact|,
 * err_bound[1] bounds max |J - J_exact| (digit truncation, dropped pairs and
 * the roundings of rho and of both recombinations).  Requires a workspace of
 * df_workspace_size bytes. */
int df_build_jk_sliced(df_ctx* ctx, const int8_t* b_dig, int planes, const int32_t* b_exp,
                       int64_t naux, int64_t nao, const double* C, int64_t nocc, double occ,
                       const double* D, double* J, double* K, double* energies,
                       double* err_bound);

/* Block screening of B (Sec. 2.1: negligible shell pairs are dropped and B
 * inherits the sparsity).  With shell blocks of `blk` consecutive basis
 * functions (blk divides 64; nao <= 4096), block (M, N) is kept iff
 * sqrt(sum_P sum_{mu in M, nu in N} B[P][mu][nu]^2) >= tau (FP64).  df_screen
 * writes mask[M][N] (uint8, 1 = kept; nblk = ceil(nao / blk)), the optional
 * norms[M][N], and chunks[mu] (uint64: bit c set iff a kept block meets row
 * mu in nu = 64c .. 64c + 63), and sets the dropped entries of B to zero IN
 * PLACE (B is modified).  Uses the context's scratch, or, for
 * nblk * nao * 8 > 8 MiB, a workspace of at least that size.
 * df_set_screening hands mask / chunks (caller-owned, kept until reset with
 * NULL) to the following df_build_jk / df_build_x calls with this nao: X and
 * the row dots of rho skip the zero nu chunks, J skips the dropped blocks.
 * The results equal the dense build of the zeroed B bit for bit (only sums of
 * exact zeros are skipped); with a B not zeroed by that mask they differ. */
int df_screen(df_ctx* ctx, double* B, int64_t naux, int64_t nao, int blk, double tau,
              uint8_t* mask, uint64_t* chunks, double* norms);
int df_set_screening(df_ctx* ctx, const uint8_t* mask, const uint64_t* chunks, int blk,
                     int64_t nao);

/* Autotuner of the launch shapes of df_build_jk for one shape at the context
 * precision and aux block size: the number of K partial groups (1, 2, 4, ...,
 * min(nblocks, 64), plus the default) and, for s <= 5 with nao % 128 == 0,
 * the k depth staged per X step (64 or 128).  Each candidate that fits the
 * current workspace runs 1 + reps full builds on the given arguments (timed
 * with HIP events; the call synchronises); the fastest is kept in the
 * context and used by every later df_build_jk / df_workspace_size of that
 * shape, precision and pblk unless df_set_k_groups fixes the groups.
 * best_groups / best_ksub / best_ms (host, may be NULL) receive the choice. */
int df_autotune(df_ctx* ctx, const double* B, const int32_t* b_exp, int64_t naux, int64_t nao,
                const double* C, int64_t nocc, double occ, const double* D, double* J, double* K,
                double* energies, double* err_bound, int reps, int* best_groups, int* best_ksub,
                double* best_ms);

/* Batched build of independent, uneven instances.  Each df_problem is one
 * df_build_jk call (dense B; b_exp may be NULL; its own slice count and
 * optional screening masks from df_screen, NULL = dense) with its own
 * outputs.  Instances are ordered by estimated cost, largest first, and
 * dealt onto `streams` (1..4) streams, each to the least-loaded one; with
 * streams > 1 the context creates worker streams (default priority) that
 * start after the work already queued on its stream and that its stream
 * waits for, so the call stays asynchronous and ordered like one build.
 * Every instance uses the autotuned shapes of df_autotune when present.
 * Workspace: df_batched_workspace_size (the sum over streams of the largest
 * instance plan on each).  The context's per-block precision must be unset. */
typedef struct df_problem {
  const double* B;
  const int32_t* b_exp;
  int64_t naux, nao, nocc;
  const double* C;
  const double* D;
  double occ;
  int slices;
  const uint8_t* screen_mask;
  const uint64_t* screen_chunks;
  int screen_blk;
  double* J;
  double* K;
  double* energies;
  double* err_bound;
} df_problem;
int df_batched_workspace_size(df_ctx* ctx, int n, const df_problem* probs, int streams,
                              size_t* bytes);
int df_build_jk_batched(df_ctx* ctx, int n, const df_problem* probs, int streams);

/* Metric Cholesky (Sec. 2.1, Eq. 2): W [n][n] symmetric positive definite is
 * overwritten in place by L (lower triangle; the upper triangle is set to 0)
 * with L L^T = W, in FP64.  A non-positive pivot sets the DF_ENOTSPD device
 * status (read with df_get_status).  Needs no workspace. */
int df_metric_cholesky(df_ctx* ctx, double* W, int64_t n);

/* Whitening of the three-index tensor (Sec. 2.1, Eq. 2): B = L^-1 T, with
 * L [naux][naux] lower triangular from df_metric_cholesky, T [naux][ncols]
 * (ncols = nao*nao for a dense tensor) and B [naux][ncols] (B must not alias
 * T).  The aux index of T is contracted with the column index of L^-1.  FP64.
 * Needs a workspace of at least naux*naux*8 bytes (it holds L^-1). */
int df_whiten(df_ctx* ctx, const double* L, int64_t naux, const double* T, int64_t ncols,
              double* B);

/* Density of closed-shell orbitals: D = occ * C C^T (D [nao][nao], C [nao][nocc])
 * in FP64 on the context stream.  Needs no workspace. */
int df_density(df_ctx* ctx, const double* C, int64_t nao, int64_t nocc, double occ, double* D);

/* Fock matrix of a closed-shell SCF iteration around the build (the SCF of
 * Sec. 4.3 in which the precision rule runs; overlap taken as the identity):
 * F = h + J - K / 2 elementwise (F[i] = (h[i] + J[i]) - 0.5 K[i]) and
 * e_one[0] = tr(D h) (device scalar; a fixed summation order), with h, J, K,
 * D, F [nao][nao] device arrays (F may alias none of the inputs).  The total
 * energy of the iteration is e_one + E_J + E_x.  Uses the context's scratch;
 * needs no workspace. */
int df_fock(df_ctx* ctx, const double* h, const double* J, const double* K, const double* D,
            int64_t nao, double* F, double* e_one);

/* Adaptive precision rule of Sec. 3.2 (Eq. 11, Table 1); host-only, no GPU work.
 *   df_rule_level(de_rel): Table 1 level for a relative energy change
 *     (>= 2e-6 -> 4, [5e-9, 2e-6) -> 3, [2e-11, 5e-9) -> 2, [7e-14, 2e-11) -> 1,
 *     below -> 0; NaN -> 4, i.e. no information).
 *   df_rule_next_level(level, e_prev, e_now): the level for the next iteration
 *     after observing E_now; dE_rel = |(E_now - E_prev) / E_now| (|dE| when
 *     E_now == 0); never returns a lower precision (a higher level) than `level`.
 *   df_rule_slices(level, fp64_below_level): INT8 split count of a level,
 *     s = ceil((m + 1) / 8) with m = 23, 31, 39, 47 for levels 4..1; 0 (native
 *     FP64) for level 0 and for every level <= fp64_below_level (the measured
 *     point where emulation stops being faster than FP64 on this GPU). */
int df_rule_level(double de_rel);
int df_rule_next_level(int level, double e_prev, double e_now);
int df_rule_slices(int level, int fp64_below_level);

/* ---- Learned slice controller (per-aux-block precision; extends the
 * per-iteration rule of Sec. 3.2 / Table 1 along the outlook of Sec. 5) ----
 * The context owns an 8 MiB device scratch for these calls (allocated by
 * df_create); calls on one context are ordered by its stream.
 *
 * df_block_stats: out[seg] = (max |A - A2|, sum (A - A2)^2) over consecutive
 *   segments of `seglen` elements of A[n] (the last one ragged); A2 may be
 *   NULL (then A alone).  nseg = ceil(n / seglen) <= 2^19.  FP64.
 * df_x_block_stats: the same over the aux blocks of X left in the workspace by
 *   the last df_build_jk of this shape (blocked layout: one segment per block
 *   of pblk aux indices); out[nblocks][2].  After an INT8 build (every block
 *   at s >= 1) the values come from what the build recorded (the maxima of
 *   its X pass, the squared sums written by its slicing of X, summed per
 *   block in a fixed order) instead of a pass over X; the sums then differ
 *   from a direct pass by rounding only.
 * df_controller_features: feat[nblocks][16] (FP32) of one iteration from
 *   bstats [nblocks][2] (df_block_stats of B per aux block), xstats
 *   [nblocks][2] (df_x_block_stats of the previous iteration), dstat[2]
 *   (D_k - D_k-1), cstat[2] (C_k), kstat[2] (K_k-1) and host_scalars[8] =
 *   {k, n_iter, dE_rel(k-1), target, nao, naux, nocc, plain-rule s}:
 *     log2 max|B_b|, log2 |B_b|_F, log10 |D_k - D_k-1|_F, k / n_iter,
 *     log10 dE_rel, log2 max|C_k|, log2 max|X_b|, log2 |X_b|_F, log2 |K_k-1|_F,
 *     log10 target, log2 nao, log2 naux, log2 nocc, s_plain / 8, b / nblocks, 1
 *   (log of 0 is written as -1100 for log2 and -330 for log10).
 * df_mlp_nparams: 5768, the FP32 parameter count, packed row-major as
 *   W1[16][64], b1[64], W2[64][64], b2[64], W3[64][8], b3[8].
 * df_mlp_forward: y[n][8] = ReLU(ReLU(x W1 + b1) W2 + b2) W3 + b3, x[n][16].
 * df_mlp_train_step: one Adam step (lr, beta1 0.9, beta2 0.999, eps 1e-8,
 *   bias-corrected with the 1-based `step`) on the masked mean squared error
 *   sum m (y - t)^2 / max(sum m, 1) over the batch rows idx[0..n-1] of
 *   x[.][16], t[.][8], mask[.][8] (idx NULL: rows 0..n-1).  params, adam_m,
 *   adam_v [5768] are updated in place; loss (device float, may be NULL)
 *   receives the batch loss before the update.  n <= 11000.  Gradient partials
 *   of 32-row tiles are summed in tile order (deterministic).
 * df_choose_slices: s_out[b] (device int32) = the smallest s in 1..8 with
 *   pred[b][s-1] <= log10(target) (compared in FP64), else 0 (native FP64).
 * df_block_partials: copies the per-block K partials K_b (lower triangles
 *   valid, without occ) of the last df_build_jk with block precision set into
 *   out[nblocks][nao][nao].
 * df_block_errors: err[b] = |occ| max_{mu >= nu} |K_b - kref_b| / kfro for the
 *   partials of the last df_build_jk with block precision set (kref as written
 *   by df_block_partials, e.g. of an all-FP64 build).
 * df_spot_check: the FP64 check of sampled blocks: for each host_blocks[i],
 *   recomputes K_b in native FP64 from B (DF_DENSE or DF_PACKED) and C and writes
 *   err[i] = |occ| max |K_b - K_b(FP64)| / kfro for the partials of the last
 *   df_build_jk with block precision set.  Needs the build's workspace. */
/* df_controller_allocate (host only, no GPU work): per-block slice counts at
 * the accuracy of one reference count.  pred [nblocks][8] (host) holds the
 * predicted log10 errors of every block for s = 1..8 (taken non-increasing in
 * s); the error budget is slack * sum_b 10^pred[b][s_ref-1], the predicted
 * error of all blocks at s_ref.  cost [8] (host, may be NULL) is the cost of
 * one block at s = 1..8 (NULL: s(s+1)/2, the digit products; a caller may
 * pass measured build times).  Starting from s = 1 everywhere, the block
 * whose move to its next count with a strictly smaller predicted error
 * removes the most error per added cost is moved, until the predicted total
 * meets the budget (or no block can improve); a move that adds no cost beats
 * every other (the largest error drop first among them).  Then every block
 * takes the largest count that costs no more than its own.  s_ref == 0 gives
 * 0 (native FP64) for all.  DF_EINVAL for a non-finite cost. */
int df_controller_allocate(const float* pred, int64_t nblocks, int s_ref, double slack,
                           const double* cost, int32_t* s_out);
int df_block_stats(df_ctx* ctx, const double* A, const double* A2, int64_t n, int64_t seglen,
                   double* out);
int df_x_block_stats(df_ctx* ctx, int64_t naux, int64_t nao, int64_t nocc, double* out);
int df_controller_features(df_ctx* ctx, const double* bstats, const double* xstats,
                           const double* dstat, const double* cstat, const double* kstat,
                           const double* host_scalars, int64_t nblocks, float* feat);
int df_mlp_nparams(void);
int df_mlp_forward(df_ctx* ctx, const float* params, const float* x, int64_t n, float* y);
int df_mlp_train_step(df_ctx* ctx, float* params, float* adam_m, float* adam_v, int64_t step,
                      const float* x, const float* t, const float* mask, const int32_t* idx,
                      int64_t n, float lr, float* loss);
int df_choose_slices(df_ctx* ctx, const float* pred, int64_t n, double target, int32_t* s_out);
int df_block_partials(df_ctx* ctx, int64_t naux, int64_t nao, int64_t nocc, double* out);
int df_block_errors(df_ctx* ctx, int64_t naux, int64_t nao, int64_t nocc, double occ,
                    const double* kref, double kfro, double* err);
int df_spot_check(df_ctx* ctx, const double* B, int layout, int64_t naux, int64_t nao,
                  const double* C, int64_t nocc, double occ, double kfro,
                  const int32_t* host_blocks, int nsample, double* err);

/* Device status word (0, DF_ENONFINITE or DF_ENOTSPD) accumulated since the last call;
 * synchronises the context stream and clears the word. */
int df_get_status(df_ctx* ctx);

/* Text of the last synchronous error of this context ("" if none). */
const char* df_last_error(const df_ctx* ctx);

/* Stages of one df_build_jk call, in launch order, for df_timing_end. */
enum df_stage {
  DF_STAGE_BEXP = 0,      /* row exponents of B (only when b_exp is NULL)        */
  DF_STAGE_PREP = 1,      /* exponents and digit planes of C                     */
  DF_STAGE_X = 2,         /* X = B C (Eq. 5), INT8 slices or FP64 MFMA, with the
                             B.D row dots of rho in the same pass over B         */
  DF_STAGE_SLICE_X = 3,   /* per-(block, mu) exponents and digits of X            */
  DF_STAGE_K = 4,         /* blocked K partials (Eq. 6): INT8 or FP64 MFMA        */
  DF_STAGE_K_REDUCE = 5,  /* sum of the block-group partials, occ, mirror         */
  DF_STAGE_RHO = 6,       /* rho (Eq. 3) from the row dots                        */
  DF_STAGE_J = 7,         /* J (Eq. 4)                                            */
  DF_STAGE_ENERGIES = 8,  /* E_J, E_x                                             */
  DF_STAGE_BOUND = 9,     /* error bound                                          */
  DF_NSTAGES = 10
};

/* Per-stage timing with HIP events on the context stream.  df_timing_begin
 * creates events for up to `max_calls` df_build_jk calls (it allocates, so
 * call it outside any timed or captured region); every following build
 * records one event per stage boundary without synchronising.
 * df_timing_end synchronises, writes the summed milliseconds per stage into
 * ms_sum[DF_NSTAGES] and the number of timed calls into *ncalls, and frees
 * the events.  Each stage's time runs from the end of the previous stage to
 * its own end on the stream. */
int df_timing_begin(df_ctx* ctx, int max_calls);
int df_timing_end(df_ctx* ctx, double* ms_sum, int* ncalls);

/* Peak probes of the device (the denominators of roofline fractions, measured
 * here instead of taken from a datasheet).  Runs one warm-up and three timed
 * launches of one probe on the context stream (synchronises; creates and
 * destroys two HIP events) and writes the rate to *rate (host):
 *   kind 0: INT8 MFMA loop (v_mfma_i32_16x16x64_i8, 8 independent chains per
 *           wave, 32 waves per CU, `iters` trips): TOP/s;
 *   kind 1: FP64 MFMA loop (v_mfma_f64_16x16x4_f64, same shape): TFLOP/s;
 *   kind 2: streaming copy of bytes / 2 into the second half of buf: GB/s of
 *           bytes read plus bytes written;
 *   kind 3: streaming read of buf: GB/s read.
 * buf: caller-owned device memory, 256-byte aligned; kinds 0/1 need
 * CUs x 16 KiB (scratch for the chain sums), kinds 2/3 at least 4 MiB (use
 * far more than the caches hold, e.g. 4 GiB).  iters 1..10^6 (kinds 2/3 ignore
 * it).  Contents of buf are overwritten. */
int df_peak_probe(df_ctx* ctx, int kind, void* buf, size_t bytes, int iters, double* rate);

/* Test hooks.
 * df_debug_build_i32: the int32 sums of the hot path itself.  Runs the INT8 X
 * and K kernels of df_build_jk at the context precision s >= 1 (uniform, no
 * per-block counts; same arguments as df_build_jk's X inputs, workspace of
 * df_workspace_size) and exports, before recombination,
 *   x_sums[g-2][P*nao + mu][i] = S_g of row (P, mu) of B and column i of C,
 *     the sum over the pairs a + b = g (g = 2..s+1, ..s+2 with extra pairs,
 *     df_set_extra_pairs) of the digit products
 *     (Sec. 3.2, Eq. 8), as accumulated by the X tiles;
 *   k_sums[g-2][b][mu][nu] = S_g of rows mu and nu of X_b (aux block b of
 *     pblk indices, nb = ceil(naux / pblk) blocks), as accumulated by the K
 *     tiles; written only where mu / 64 >= nu / 64 (the lower 64 x 64 tiles
 *     the K kernel forms).
 * df_debug_slice_gemm_i32: the exact int32 product of every kept slice pair of
 * given digit planes, formed by a plain kernel on the same MFMA instruction
 * (v_mfma_i32_16x16x64_i8; not the tiles of the hot path).  a_dig [s][m][k]
 * and b_dig [s][k][n] are int8 digit planes; partials[p][m][n] receives
 * sum_k a_dig[a-1][.][k] * b_dig[b-1][k][.] for the p-th pair (a, b) in the
 * order a = 1..s, b = 1..s+1-a.  Needs k < 131072 (128^2 k < 2^31) and a
 * workspace of at least s*M*Kp (rounded up to 256) + s*N*Kp bytes, with
 * M, N, Kp = m, n, k rounded up to multiples of 64. */
int df_debug_build_i32(df_ctx* ctx, const double* B, int layout, int64_t naux, int64_t nao,
                       const int32_t* b_exp, const double* C, int64_t nocc, int32_t* x_sums,
                       int32_t* k_sums);
int df_debug_slice_gemm_i32(df_ctx* ctx, const int8_t* a_dig, const int8_t* b_dig, int64_t m,
                            int64_t n, int64_t k, int s, int32_t* partials);

#ifdef __cplusplus
}
#endif

#endif /* DFJK_H */
