// Internal declarations shared by the HIP translation units of libdfjk.
// gfx950 (CDNA4) only: 64-wide wavefronts, INT8 and FP64 MFMA.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

namespace dfjk {

constexpr int kWave = 64;
// LDS one gfx950 workgroup may allocate (bytes); every kernel with a large
// static LDS footprint checks it at compile time.  No launch uses dynamic LDS.
constexpr int kLdsLimit = 160 * 1024;
constexpr int kMaxSlices = 8;
constexpr int kStatusNonFinite = 1;
constexpr int kStatusNotSpd = 2;

// Exponent e with 2^(e-1) <= m < 2^e for m > 0, and 0 for m == 0.
__device__ __forceinline__ int exp_of_max(double m) {
  int e = 0;
  if (m != 0.0) (void)frexp(m, &e);
  return e;
}

// Balanced base-256 digits of N = trunc(a * 2^(62 - e)), |N| < 2^62, packed in
// one word: byte 7 holds d_1 (most significant, |d_1| <= 64), byte 0 holds d_8.
// N is formed exactly in FP64 (power-of-two scaling, trunc) and split into its
// high and low 32-bit halves (floor of y / 2^32, then the exact remainder).
// Adding 0x80 to each of the seven low bytes and flipping their top bit turns
// the two's-complement bytes of N into the balanced digits in [-128, 127]
// (each low byte u becomes u - 128 once the carries of the +0x80 have moved
// up).  Requires |a| < 2^e (e is the exponent of the row maximum).
// digit_word_offset stops before the flip (its seven low bytes still carry the
// 0x80 offset), for callers that flip whole packed words later.
__device__ __forceinline__ uint64_t digit_word_offset(double a, int e) {
  const double y = trunc(ldexp(a, 62 - e));
  const double yh = floor(y * 0x1p-32);
  const double yl = fma(-yh, 0x1p32, y);
  const unsigned long long n =
      ((unsigned long long)(unsigned int)(int)yh << 32) | (unsigned long long)(unsigned int)yl;
  return n + 0x0080808080808080ull;
}
__device__ __forceinline__ uint64_t digit_word(double a, int e) {
  return digit_word_offset(a, e) ^ 0x0080808080808080ull;
}

// Digit k (1-based, 1 = most significant) of a digit word, as a byte.
__device__ __forceinline__ uint32_t digit_byte(uint64_t w, int k) {
  return (uint32_t)(w >> (8 * (8 - k))) & 0xffu;
}

// Error-bound factor of one emulated product over k terms (slices s >= 1), or
// the FP64 dot-product factor gamma_k (s == 0):
//   |Z - Z_hat| <= k 2^(e_r + f_c) kappa.
// s >= 1: slicing of both operands (2 eps + eps^2, eps the largest dropped
// tail of a balanced base-256 expansion plus the 62-bit truncation), the digit
// pairs with a + b >= s + 2 + extra that are not formed (2s + 1 - g pairs of
// weight 2^(18 - 8g) at each g), and the s + extra - 1 FP64 roundings of the
// recombination.  extra (the anti-diagonals kept beyond s + 1) is clamped to
// 0..s-1.
__host__ __device__ inline double kappa_of(int s, int64_t k, int extra = 0) {
  const double u = 0x1p-53;
  if (s == 0) {
    const double ku = (double)k * u;
    return ku / (1.0 - ku);
  }
  const int ex = extra < 0 ? 0 : (extra > s - 1 ? s - 1 : extra);
  const double eps = (128.0 / 255.0) * ldexp(1.0, 2 - 8 * s) * (1.0 - ldexp(1.0, -8 * (8 - s))) +
                     0x1p-62;
  double dropped = 0.0;
  for (int g = s + 2 + ex; g <= 2 * s; ++g)
    dropped += (double)(2 * s + 1 - g) * ldexp(1.0, 18 - 8 * g);
  const int nadd = s + ex - 1;
  const double rounding = nadd * u * 1.016 * pow(1.0 + u, (double)(nadd + 1));
  return 2.0 * eps + eps * eps + dropped + rounding;
}

// Byte offset of 16-byte unit `unit` (0..3) of a 64-byte LDS row: the units are
// XOR-swizzled with bits 1..2 of the row, so that the 16 rows of an MFMA
// fragment read (16 lanes, one unit each) spread over all LDS banks.
__device__ __forceinline__ int swz(int row, int unit) { return (unit ^ ((row >> 1) & 3)) << 4; }

// Workgroups are handed to the 8 XCDs of the chip round-robin by linear id,
// and each XCD has its own L2.  xcd_order(id, n) renumbers the n workgroups of a
// launch so that XCD x receives the consecutive logical range
// [x n / 8, (x + 1) n / 8) (a bijection on [0, n)): logically adjacent work
// items that share operands then meet in one L2.
__device__ __forceinline__ int64_t xcd_order(int64_t id, int64_t n) {
  const int64_t x = id & 7, i = id >> 3, q = n >> 3, r = n & 7;
  return x * q + (x < r ? x : r) + i;
}

// Set bits of a chunk mask: the first one, and the first one above c (-1: none).
__device__ __forceinline__ int first_bit(unsigned long long m) {
  return m ? __ffsll((unsigned long long)m) - 1 : -1;
}
__device__ __forceinline__ int next_bit(unsigned long long m, int c) {
  const unsigned long long r = c >= 63 ? 0ull : (m >> (c + 1)) << (c + 1);
  return r ? __ffsll((unsigned long long)r) - 1 : -1;
}

// Union over the 64 rows m0 .. m0 + 63 (rows < M; row r is basis row r % nao)
// of the per-row masks of 64-wide nu chunks that meet a kept block of the
// screened B, folded to 128-wide chunks when KSUB == 2.  Every thread of the
// workgroup must call it (it synchronises); wave 0 does the reduction.
template <int KSUB>
__device__ __forceinline__ unsigned long long tile_chunks(const unsigned long long* cmask,
                                                          int64_t m0, int64_t M, int nao, int w,
                                                          int l) {
  __shared__ unsigned long long tmask;
  if (w == 0) {
    const int64_t row = m0 + l;
    unsigned long long m = row < M ? cmask[row % nao] : 0ull;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) m |= __shfl_xor(m, off);
    if (l == 0) tmask = m;
  }
  __syncthreads();
  unsigned long long live = tmask;
  if (KSUB == 2) {
    unsigned long long f = 0;
    for (int c = 0; c < 32; ++c)
      if ((live >> (2 * c)) & 3ull) f |= 1ull << c;
    live = f;
  }
  return live;
}

__device__ __forceinline__ double abs_max_bits_to_double(unsigned long long b) {
  return __longlong_as_double((long long)b);
}

}  // namespace dfjk

// ---------------------------------------------------------------------------
// Kernel launchers (each defined next to its kernels); all enqueue on `st`.
// ---------------------------------------------------------------------------
namespace dfjk {

// slicing.hip
hipError_t launch_row_exp(hipStream_t st, const double* A, int64_t rows, int64_t cols,
                          int64_t lda, int32_t* e, int* status);
// Row exponents of a packed B ([naux][nao (nao + 1) / 2], lower triangles by rows).
hipError_t launch_row_exp_packed(hipStream_t st, const double* B, int64_t naux, int nao,
                                 int32_t* e, int* status);
hipError_t launch_col_exp(hipStream_t st, const double* C, int64_t nao, int64_t nocc,
                          int32_t* f, int* status);
hipError_t launch_slice_rows(hipStream_t st, const double* A, int64_t rows, int64_t cols,
                             int64_t lda, int s, const int32_t* e, int8_t* digits);
// C digits in the operand layout of the INT8 X product: [s][ncp][kp], k in the
// slot order of the B-tile loader (natural = 0) or in natural order, zero padded.
hipError_t launch_slice_c(hipStream_t st, const double* C, int64_t nao, int64_t nocc, int s,
                          const int32_t* f, int ncp, int kp, int natural, int8_t* dC);
hipError_t launch_fill_u64(hipStream_t st, unsigned long long* p, int64_t n,
                           unsigned long long v);
hipError_t launch_fill_i32(hipStream_t st, int* p, int64_t n, int v);

// int8_gemm.hip
// X layout 0: [naux*nao][nocc]; 1: blocked, X_b rows mu over (P - P0, i) with
// block stride pblk * nocc.  D / rowdot optional: rowdot[P*nao + mu] = B row . D row.
hipError_t launch_x_int8(hipStream_t st, int s, const double* B, int64_t naux, int nao,
                         const int32_t* b_exp, const int8_t* dC, int ncp, int kp,
                         const int32_t* f_col, int nocc, double* X, int xlayout,
                         unsigned long long* xmax, int pblk, const double* D, double* rowdot,
                         const unsigned long long* cmask = nullptr, int ksub = 0,
                         int32_t* dbg = nullptr, int packed = 0, int extra = 0);
// (ksub: k depth per LDS stage, 1 = 64, 2 = 128 where s <= 5 and nao % 128 == 0,
// 0 = the default choice.  dbg, a test export: [s][naux*nao][nocc] int32
// anti-diagonal sums g = 2..s+1 of the tiles.  packed: B as [naux][nao(nao+1)/2],
// the lower triangle of each B_P by rows (no screening masks; 64-wide chunks).
// extra: anti-diagonals kept beyond a + b = s + 1 (0 or 1; 64-wide chunks).)
// X in the blocked layout.  xss (optional): the sums of squares of X in
// slots of 16 rows x 64 values, [nb][kbp / 64][nao_pad / 16] (slot order of
// the block's X digits: step, then rows).
hipError_t launch_slice_x(hipStream_t st, int s, const double* Xb, int64_t naux, int nao,
                          int nocc, int pblk, int nao_pad, int kbp,
                          const unsigned long long* xmax, int32_t* F, int8_t* Xd,
                          double* xss = nullptr);
// out[b] = (max over mu of the |X| maxima xmax[b][mu], the sum of block b's
// nslot slots of xss in a fixed order) for b < nb.
hipError_t launch_xstats_from(hipStream_t st, const unsigned long long* xmax, const double* xss,
                              int nb, int nao, int64_t nslot, double* out);
// Workgroups of the INT8 K kernel for s slices that one CU holds at once.
int k_int8_resident(int s);
// dbg (test export, may be null): [s][nb][nao][nao] int32 anti-diagonal sums
// per aux block, written where mu / 64 >= nu / 64 (the lower tiles).
hipError_t launch_k_int8(hipStream_t st, int s, const int8_t* Xd, const int32_t* F, int nb,
                         int nao, int nao_pad, int kbp, int groups, double* Kp,
                         int32_t* dbg = nullptr, int extra = 0);
hipError_t launch_debug_pairs(hipStream_t st, int s, const int8_t* a_dig, const int8_t* b_dig,
                              int64_t m, int64_t n, int64_t k, int8_t* ws_a, int8_t* ws_b,
                              int32_t* partials);

// fp64_gemm.hip
hipError_t launch_x_fp64(hipStream_t st, const double* B, int64_t naux, int nao,
                         const double* C, int nocc, double* X, int xlayout,
                         unsigned long long* xmax, int pblk, const double* D, double* rowdot,
                         const unsigned long long* cmask = nullptr, int packed = 0);
// X in the blocked layout.
hipError_t launch_k_fp64(hipStream_t st, const double* Xb, int64_t naux, int nao, int nocc,
                         int pblk, int nb, int groups, double* Kp);
hipError_t launch_xmax_to_exp(hipStream_t st, const unsigned long long* xmax, int64_t n,
                              int32_t* F);

// metric.hip (Sec. 2.1, Eq. 2)
hipError_t launch_cholesky(hipStream_t st, double* A, int64_t n, int* status);
hipError_t launch_tri_inverse(hipStream_t st, const double* L, int64_t n, double* Linv);
hipError_t launch_whiten(hipStream_t st, const double* Linv, int64_t naux, const double* T,
                         int64_t ncols, double* Bout);
hipError_t launch_density(hipStream_t st, const double* C, int64_t nao, int64_t nocc, double occ,
                          double* D);

// jk.hip
hipError_t launch_rho(hipStream_t st, const double* B, int64_t naux, int nao, const double* D,
                      double* rho);
// rho_P = sum_mu rowdot[P*nao + mu] (fixed order).
hipError_t launch_rho_reduce(hipStream_t st, const double* rowdot, int64_t naux, int nao,
                             double* rho);
// With smask ([nblk][nblk] kept shell blocks of size blk), dropped blocks are
// not read (they are zero in the screened B).
hipError_t launch_j(hipStream_t st, const double* B, int64_t naux, int nao, const double* rho,
                    int jsplit, double* Jp, double* J, const uint8_t* smask = nullptr, int blk = 8,
                    int packed = 0);
hipError_t launch_k_reduce(hipStream_t st, const double* Kp, int groups, int nao, double occ,
                           double* K);
// F = h + J - K / 2 and e_one = tr(D h) (scratch: 256 doubles).
hipError_t launch_fock(hipStream_t st, const double* h, const double* J, const double* K,
                       const double* D, int64_t nao, double* F, double* scratch, double* e_one);
// scratch: 2 * 256 doubles.
hipError_t launch_energies(hipStream_t st, const double* rho, int64_t naux, const double* D,
                           const double* K, int nao, double* scratch, double* energies);
// Error bound of the blocked K: kappa1 / kappa2 from the host, or, with sblk
// (device [nb] slice counts) given, each block's own factors.
hipError_t launch_bound(hipStream_t st, const int32_t* b_exp, const int32_t* f_col, int nocc,
                        const int32_t* F, int fstride, int64_t naux, int nao, int pblk, int nb,
                        double kappa1, double kappa2_full, double kappa2_last, double occ,
                        const int32_t* sblk, double* scratch, double* err_bound, int extra = 0);


// sliced.hip: the mode with B held as digit planes [planes][naux*nao][ldk]
// (ldk = nao rounded up to 64, zero padded).
// packed: A is a packed B (rows P cols + mu), see k_slice_planes.
hipError_t launch_slice_planes(hipStream_t st, const double* A, int64_t rows, int cols, int ldk,
                               const int32_t* e, int planes, int8_t* dig, int packed = 0);
// X (blocked layout) from the B planes and the natural-order C digits; with
// Dd / d_exp, rowdot[P*nao + mu] = the emulated B row . D row.
hipError_t launch_x_dig(hipStream_t st, int s, const int8_t* Bd, int64_t bplane, int64_t naux,
                        int nao, int ldk, const int32_t* b_exp, const int8_t* dC, int ncp,
                        const int32_t* f_col, int nocc, double* X, unsigned long long* xmax,
                        int pblk, const int8_t* Dd, const int32_t* d_exp, double* rowdot);
// rho (mu ascending) and its per-P error bound.
hipError_t launch_rho_seq(hipStream_t st, const double* rowdot, const int32_t* b_exp,
                          const int32_t* d_exp, int64_t naux, int nao, double kap_row,
                          double kap_sum, double* rho, double* drho);
// J from the B planes; jbound receives the Coulomb error bound (as double bits).
hipError_t launch_j_dig(hipStream_t st, int s, const int8_t* Bd, int64_t bplane, int ldk,
                        const double* rho, const double* drho, const int32_t* b_exp, int64_t naux,
                        int nao, int naux_pad, int nsplit, double kap_j, int32_t* h, int8_t* wd,
                        unsigned long long* Sj, unsigned long long* jbound, double* J);

// screen.hip: shell-block norms over all P (part: nsplit * nblk * nao doubles),
// mask (keep iff norm >= tau), zeroing of the dropped blocks of B in place,
// per-row chunk masks (64-wide nu chunks, nao <= 4096); norms may be null.
hipError_t launch_screen(hipStream_t st, double* B, int64_t naux, int nao, int blk, double tau,
                         int nsplit, double* part, double* norms, uint8_t* mask,
                         unsigned long long* chunks);

// peak.hip: device peak probes.  kind 0: INT8 MFMA loop, 1: FP64 MFMA loop
// (iters loop trips; buf >= ncu * 8 * 256 * 8 bytes), 2: streaming copy of
// bytes / 2 into the other half, 3: streaming read.  *work receives the ops
// (0, 1) or bytes moved (2, 3) of the launch.
hipError_t launch_peak(hipStream_t st, int kind, int ncu, void* buf, size_t bytes, int iters,
                       double* work);

// controller.hip (the per-block slice controller)
struct CtlScalars {  // host scalars of one iteration, passed by value
  double iteration, n_iter, de_rel, target, nao, naux, nocc, plain_s;
};
int mlp_nparam();
// out[seg] = (max |A - A2|, sum (A - A2)^2) over segments of seglen elements (A2 may be null);
// in the last segment only the first last_valid of every rowlen elements count;
// partial: nseg * nsplit * 2 doubles.
hipError_t launch_seg_stats(hipStream_t st, const double* A, const double* A2, int64_t n,
                            int64_t seglen, int64_t rowlen, int64_t last_valid, double* partial,
                            int nsplit, double* out);
hipError_t launch_features(hipStream_t st, const double* bstats, const double* xstats,
                           const double* dstat, const double* cstat, const double* kstat,
                           const CtlScalars& sc, int nb, float* feat);
hipError_t launch_mlp_forward(hipStream_t st, const float* prm, const float* x, int64_t n, float* y);
// gpart: ceil(n / 32) * (nparam + 1) floats; cnt: 1 float.
hipError_t launch_mlp_train(hipStream_t st, float* prm, float* m1, float* m2, int64_t step,
                            const float* x, const float* t, const float* mask, const int32_t* idx,
                            int64_t n, float lr, float* gpart, float* cnt, float* loss);
hipError_t launch_choose(hipStream_t st, const float* pred, int64_t n, double target, int32_t* s);
hipError_t launch_block_err(hipStream_t st, const double* Kp, const double* Kref, int nao,
                            double scale, double* err);
hipError_t launch_copy_f64(hipStream_t st, const double* a, int64_t n, double* b);

}  // namespace dfjk
