// Sliced mode of the build: B is kept as INT8 digit planes (sliced once per B;
// any prefix of the planes serves every level), and X, rho and J are all formed
// from those digits; FP64 remains in the recombinations and the energies.
//   X   = B C               (Eq. 5): INT8 MFMA, A fragments read from the planes
//   rho = sum_{mu,nu} B D   (Eq. 3): per row (P, mu), an INT8 dot (v_dot4) of the
//                                  row's digits with the digits of D's row mu on
//                                  the same fragments, recombined in FP64, then
//                                  summed over mu in ascending order
//   J   = sum_P rho_P B_P   (Eq. 4): w[P, mu] = rho_P 2^e[P, mu] sliced over P for
//                                  each mu; INT8 dots with the B digits over P
//                                  (lower triangle), mirrored
// Digit planes share one row stride `ldk` (the row length rounded up to 64
// bytes, zero padded), so every 16-byte fragment load stays inside its row.
#include "dfjk_internal.h"

namespace dfjk {
namespace {

__device__ __forceinline__ uint32_t pack4(uint64_t w0, uint64_t w1, uint64_t w2, uint64_t w3,
                                          int k) {
  return digit_byte(w0, k) | (digit_byte(w1, k) << 8) | (digit_byte(w2, k) << 16) |
         (digit_byte(w3, k) << 24);
}

// dig[a][r][ldk] = digit a + 1 of A[r][c] (row exponent e[r]); columns c >= cols
// are zero.  One thread per 16 output bytes of a row.  packed != 0: A is a
// packed B (rows r = P cols + mu of B_P; B_P stored as its lower triangle by
// rows, element (mu, c) at max (max + 1) / 2 + min), read element by element.
__global__ __launch_bounds__(256) void k_slice_planes(const double* __restrict__ A, int64_t rows,
                                                      int cols, int ldk,
                                                      const int32_t* __restrict__ e, int planes,
                                                      int8_t* __restrict__ dig, int packed) {
  const int nc = ldk / 16;
  const int64_t total = rows * nc;
  const int64_t plane = rows * (int64_t)ldk;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = idx / nc;
    const int c0 = (int)(idx - r * nc) * 16;
    const double* src = A + r * cols + c0;
    const int er = e[r];
    uint64_t wd[16];
    if (packed) {
      const int64_t P = r / cols;
      const int mu = (int)(r - P * cols);
      const double* bp = A + P * ((int64_t)cols * (cols + 1) / 2);
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int c = c0 + j;
        const int64_t o = c <= mu ? (int64_t)mu * (mu + 1) / 2 + c : (int64_t)c * (c + 1) / 2 + mu;
        wd[j] = c < cols ? digit_word(bp[o], er) : 0ull;
      }
    } else if (c0 + 16 <= cols && (cols & 1) == 0) {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const double2 p = *reinterpret_cast<const double2*>(src + 2 * j);
        wd[2 * j] = digit_word(p.x, er);
        wd[2 * j + 1] = digit_word(p.y, er);
      }
    } else {
#pragma unroll
      for (int j = 0; j < 16; ++j) wd[j] = c0 + j < cols ? digit_word(src[j], er) : 0ull;
    }
    int8_t* dst = dig + r * ldk + c0;
    for (int a = 0; a < planes; ++a) {
      i32x4 pk;
      pk[0] = (int)pack4(wd[0], wd[1], wd[2], wd[3], a + 1);
      pk[1] = (int)pack4(wd[4], wd[5], wd[6], wd[7], a + 1);
      pk[2] = (int)pack4(wd[8], wd[9], wd[10], wd[11], a + 1);
      pk[3] = (int)pack4(wd[12], wd[13], wd[14], wd[15], a + 1);
      *reinterpret_cast<i32x4*>(dst + a * plane) = pk;
    }
  }
}

// 16 bytes per lane from a buffer resource (byte offset voff + soff) straight
// into LDS: lane i of the wave writes bytes 16 i .. 16 i + 15 after the
// wave-uniform LDS address lds_dst.  Completion is counted by vmcnt.
__device__ __forceinline__ void copy16_lds(__amdgpu_buffer_rsrc_t r, void* lds_dst, int voff,
                                           int soff) {
  __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (__attribute__((address_space(3))) void*)lds_dst, 16,
                                           voff, soff, 0, 0);
}

// X = B C from the B digit planes, both operands copied from memory straight
// into LDS (buffer loads to LDS: no per-value VALU work).  Tile: 64 rows x NT
// columns (NT = 16 NFW NH); wave w owns rows 16 (w & 3) .. +15 and column
// fragments [NFW (w >> 2), +NFW).  A stage holds, for one 64-wide k chunk, the
// S planes of the tile's rows [64][64 B] and of its C columns [NT][64 B]; the
// four 16-byte units of row (or column) r sit in the slots unit ^ ((r >> 1) & 3)
// (the swizzle is made by choosing which unit each lane copies: one copy
// instruction fills 16 rows, lane l row l >> 2, slot l & 3).  Two stages, each
// its own __shared__ array (so that the compiler can tell the stage being
// filled from the one being read): after the barrier of chunk c the copies of
// chunk c + 1 are issued into the stage chunk c - 1 used, and land while chunk
// c is multiplied; one barrier per chunk.  (Measured: a third stage, which
// leaves one workgroup per CU where two stages leave two, was slower at s = 3
// and no faster at s = 5.)  Lane (q, r) of an A fragment holds the 16 bytes
// k0 + 16 q .. +15 of its row, natural k order (the C digits are in natural
// order too).  With D digits given, waves of half 0 of the first column tile
// also accumulate the row dots of rho per anti-diagonal with v_dot4 on their
// A fragments and D fragments read from memory (exact int32), then recombine
// them in FP64.
template <int S, int NFW, int NH>
__global__ __launch_bounds__(256 * NH) void k_x_dig(
    const int8_t* __restrict__ Bd, int64_t bplane, int64_t M, int ldk,
    const int32_t* __restrict__ b_exp, const int8_t* __restrict__ dC, int ncp,
    const int32_t* __restrict__ f_col, int nocc, double* __restrict__ X,
    unsigned long long* __restrict__ xmax, int nao, int pblk,
    const int8_t* __restrict__ Dd, const int32_t* __restrict__ d_exp, double* __restrict__ rowdot) {
  constexpr int NF = NFW * NH, NT = 16 * NF, NW = 4 * NH;
  constexpr int ACOPY = 4 * S, CCOPY = NF * S;  // copies of a chunk (16 rows / columns each)
  constexpr int PA = (ACOPY + NW - 1) / NW, PC = (CCOPY + NW - 1) / NW;
  constexpr int ASZ = S * 64 * 64, CSZ = S * NT * 64;
  __shared__ __attribute__((aligned(16))) int8_t As0[ASZ];
  __shared__ __attribute__((aligned(16))) int8_t As1[ASZ];
  __shared__ __attribute__((aligned(16))) int8_t Cs0[CSZ];
  __shared__ __attribute__((aligned(16))) int8_t Cs1[CSZ];
  static_assert(2 * (ASZ + CSZ) <= kLdsLimit, "X stages exceed LDS");
  const int t = threadIdx.x, w = t >> 6, l = t & 63, q = l >> 4, r16 = l & 15;
  const int wr = w & 3, half = w >> 2;
  // tiles in the logical order (row tile, column tile), handed to the XCDs
  // in contiguous ranges: the column tiles of one row tile share its B digits
  // in one L2, and neighbouring row tiles (consecutive P at one mu tile when
  // nao is a multiple of 64) share the rows of D
  const int ncol = ncp / NT;
  const int64_t lid = xcd_order(blockIdx.x, gridDim.x);
  const int64_t rt = lid / ncol;
  const int ct = (int)(lid - rt * ncol);
  int64_t m0 = rt * 64;
  if (nao % 64 == 0) {
    const int64_t naux = M / nao;
    const int64_t mt = rt / naux, P = rt - mt * naux;
    m0 = P * nao + mt * 64;
  }
  const int n0 = ct * NT;
  const int64_t arow = m0 + wr * 16 + r16;
  const bool aok = arow < M;
  const bool want_rd = Dd != nullptr && ct == 0 && half == 0;
  const int mu_a = aok ? (int)(arow % nao) : 0;
  const int8_t* dsrc = (Dd ? Dd : Bd) + (int64_t)mu_a * ldk + q * 16;
  const int64_t dplane = (int64_t)nao * ldk;
  const int nch = ldk / 64;

  // this wave's copies: A copy j = w + NW i (plane j >> 2, rows 16 (j & 3)
  // .. +15 of the tile), C copy j = w + NW i (plane j / NF, columns 16 (j % NF)
  // .. +15); lane l copies row (column) l >> 2 of the group, global unit
  // (l & 3) ^ ((l >> 3) & 3), into slot l & 3
  const int cvoff = (l >> 2) * ldk + (((l & 3) ^ ((l >> 3) & 3)) << 4);
  __amdgpu_buffer_rsrc_t crA[PA], crC[PC];
  int cdA[PA], cdC[PC];
#pragma unroll
  for (int i = 0; i < PA; ++i) {
    const int j = w + NW * i;
    const int jj = j < ACOPY ? j : 0;
    const int a = jj >> 2, grp = jj & 3;
    const int64_t r0 = m0 + 16 * grp;
    const int64_t nrow = M - r0 < 0 ? 0 : (M - r0 > 16 ? 16 : M - r0);
    crA[i] = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<int8_t*>(Bd + a * bplane + (nrow ? r0 : 0) * (int64_t)ldk), (short)0,
        (int)(nrow * ldk), 0x00020000);
    cdA[i] = (a * 64 + 16 * grp) * 64;
  }
#pragma unroll
  for (int i = 0; i < PC; ++i) {
    const int j = w + NW * i;
    const int jj = j < CCOPY ? j : 0;
    const int a = jj / NF, grp = jj - a * NF;
    crC[i] = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<int8_t*>(dC + ((int64_t)a * ncp + n0 + 16 * grp) * ldk), (short)0, 16 * ldk,
        0x00020000);
    cdC[i] = (a * NT + 16 * grp) * 64;
  }
#define DFJK_XD_COPY(AS, CS, CC)                                                            \
  {                                                                                         \
    _Pragma("unroll") for (int i = 0; i < PA; ++i) {                                        \
      if (w + NW * i < ACOPY) copy16_lds(crA[i], (AS) + cdA[i], cvoff, (CC) * 64);          \
    }                                                                                       \
    _Pragma("unroll") for (int i = 0; i < PC; ++i) {                                        \
      if (w + NW * i < CCOPY) copy16_lds(crC[i], (CS) + cdC[i], cvoff, (CC) * 64);          \
    }                                                                                       \
  }

  i32x4 acc[S][NFW];
#pragma unroll
  for (int g = 0; g < S; ++g)
#pragma unroll
    for (int f = 0; f < NFW; ++f) acc[g][f] = i32x4{0, 0, 0, 0};
  int rdi[S];
#pragma unroll
  for (int g = 0; g < S; ++g) rdi[g] = 0;
  i32x4 dcur[S];
#pragma unroll
  for (int b = 0; b < S; ++b) dcur[b] = i32x4{0, 0, 0, 0};
#define DFJK_XD_LOADD(DST, CC)                                                              \
  {                                                                                         \
    if (want_rd) {                                                                          \
      _Pragma("unroll") for (int b = 0; b < S; ++b) DST[b] =                                \
          *reinterpret_cast<const i32x4*>(dsrc + b * dplane + (CC) * 64);                   \
    }                                                                                       \
  }
  // chunk CC (stage AS, CS): wait for its copies, meet at the barrier, load
  // chunk CC's D rows (used after the MFMAs), start the copies of chunk CC + 1
  // into the stage chunk CC - 1 used (ASN, CSN), then multiply
#define DFJK_XD_STEP(AS, CS, ASN, CSN, CC)                                                  \
  {                                                                                         \
    const int cc = (CC);                                                                    \
    asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)\n\ts_barrier" ::: "memory");             \
    DFJK_XD_LOADD(dcur, cc)                                                                 \
    if (cc + 1 < nch) DFJK_XD_COPY(ASN, CSN, cc + 1)                                        \
    const int8_t* As = (AS);                                                                \
    const int8_t* Cs = (CS);                                                                \
    const int arw = wr * 16 + r16;                                                          \
    i32x4 acur[S];                                                                          \
    _Pragma("unroll") for (int a = 0; a < S; ++a) acur[a] =                                 \
        *reinterpret_cast<const i32x4*>(As + (a * 64 + arw) * 64 + swz(arw, q));            \
    _Pragma("unroll") for (int f = 0; f < NFW; ++f) {                                       \
      const int col = (half * NFW + f) * 16 + r16;                                          \
      _Pragma("unroll") for (int b = 0; b < S; ++b) {                                       \
        const i32x4 bf =                                                                    \
            *reinterpret_cast<const i32x4*>(Cs + (b * NT + col) * 64 + swz(col, q));        \
        _Pragma("unroll") for (int a = 0; a < S - b; ++a) acc[a + b][f] =                   \
            __builtin_amdgcn_mfma_i32_16x16x64_i8(acur[a], bf, acc[a + b][f], 0, 0, 0);     \
      }                                                                                     \
    }                                                                                       \
    if (want_rd) {                                                                          \
      _Pragma("unroll") for (int a = 0; a < S; ++a)                                         \
      _Pragma("unroll") for (int b = 0; b < S - a; ++b) {                                   \
        int v = rdi[a + b];                                                                 \
        _Pragma("unroll") for (int j = 0; j < 4; ++j) v =                                   \
            __builtin_amdgcn_sdot4(acur[a][j], dcur[b][j], v, false);                       \
        rdi[a + b] = v;                                                                     \
      }                                                                                     \
    }                                                                                       \
  }

  // prologue: the copies of chunk 0; a step's copies go into the stage the
  // previous step read
  DFJK_XD_COPY(As0, Cs0, 0)
  for (int c = 0; c < nch; c += 2) {
    DFJK_XD_STEP(As0, Cs0, As1, Cs1, c)
    if (c + 1 < nch) DFJK_XD_STEP(As1, Cs1, As0, Cs0, c + 1)
  }
#undef DFJK_XD_STEP
#undef DFJK_XD_LOADD
#undef DFJK_XD_COPY

  if (want_rd) {
    // exact sums over the four lane groups of the row, then its recombination
#pragma unroll
    for (int g = 0; g < S; ++g) {
      rdi[g] += __shfl_xor(rdi[g], 16);
      rdi[g] += __shfl_xor(rdi[g], 32);
    }
    if (q == 0 && aok) {
      const int base = b_exp[arow] + d_exp[mu_a] + 4;
      double z = 0.0;
#pragma unroll
      for (int g = S + 1; g >= 2; --g) z += ldexp((double)rdi[g - 2], base - 8 * g);
      rowdot[arow] = z;
    }
  }

#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int64_t row = m0 + wr * 16 + q * 4 + r;
    const bool vr = row < M;
    const int er = vr ? b_exp[row] : 0;
    const int64_t P = vr ? row / nao : 0;
    const int mu = (int)(row - P * nao);
    const int64_t b = P / pblk;
    double* xrow = X + (((b * nao + mu) * pblk + (P - b * pblk)) * (int64_t)nocc);
    double rmax = 0.0;
#pragma unroll
    for (int f = 0; f < NFW; ++f) {
      const int col = n0 + (half * NFW + f) * 16 + r16;
      if (vr && col < nocc) {
        const int base = er + f_col[col] + 4;
        double z = 0.0;
#pragma unroll
        for (int g = S + 1; g >= 2; --g) z += ldexp((double)acc[g - 2][f][r], base - 8 * g);
        xrow[col] = z;
        rmax = fmax(rmax, fabs(z));
      }
    }
#pragma unroll
    for (int off = 1; off < 16; off <<= 1) rmax = fmax(rmax, __shfl_xor(rmax, off));
    if (r16 == 0 && vr)
      atomicMax(&xmax[b * nao + mu], (unsigned long long)__double_as_longlong(rmax));
  }
}

// rho_P = sum_mu rowdot[P nao + mu] with mu ascending (one thread per P), and
// the bound on |rho_P - rho_hat_P|: the emulated row dots (nao terms each,
// exponents e_B + g) plus the nao - 1 roundings of the mu sum.  A workgroup
// takes 64 consecutive P; 64 x 64 tiles of the row dots and exponents are read
// coalesced into LDS and each of 64 threads walks its row of the tile.
__global__ __launch_bounds__(256) void k_rho_seq(const double* __restrict__ rowdot,
                                                 const int32_t* __restrict__ b_exp,
                                                 const int32_t* __restrict__ d_exp, int64_t naux,
                                                 int nao, double kap_row, double kap_sum,
                                                 double* __restrict__ rho,
                                                 double* __restrict__ drho) {
  __shared__ double tr[64][65];
  __shared__ int te[64][65];
  const int t = threadIdx.x;
  const int64_t P0 = (int64_t)blockIdx.x * 64;
  double a = 0.0, sabs = 0.0, srow = 0.0;
  for (int mu0 = 0; mu0 < nao; mu0 += 64) {
    __syncthreads();
    for (int e = t; e < 64 * 64; e += 256) {
      const int pl = e >> 6, ml = e & 63;
      const int64_t P = P0 + pl;
      const int mu = mu0 + ml;
      const bool ok = P < naux && mu < nao;
      tr[pl][ml] = ok ? rowdot[P * nao + mu] : 0.0;
      te[pl][ml] = ok ? b_exp[P * nao + mu] + d_exp[mu] : 0;
    }
    __syncthreads();
    if (t < 64) {
      const int mend = nao - mu0 < 64 ? nao - mu0 : 64;
      for (int ml = 0; ml < mend; ++ml) {
        const double v = tr[t][ml];
        a += v;
        sabs += fabs(v);
        srow += ldexp(1.0, te[t][ml]);
      }
    }
  }
  if (t < 64 && P0 + t < naux) {
    rho[P0 + t] = a;
    drho[P0 + t] = (double)nao * kap_row * srow + kap_sum * sabs;
  }
}

// For one mu: w[P] = rho_P 2^e[P, mu]; h_mu = exponent of max_P |w|; the digit
// planes wd[a][mu][P] (P padded to naux_pad with zeros); and the Coulomb error
// bound at mu, naux 2^h kappa(naux) + sum_P drho_P 2^e[P, mu], max-ed into
// jbound (non-negative doubles compare as their bit patterns).
__global__ __launch_bounds__(256) void k_slice_w(const double* __restrict__ rho,
                                                 const double* __restrict__ drho,
                                                 const int32_t* __restrict__ b_exp, int64_t naux,
                                                 int nao, int S, int naux_pad, double kap_j,
                                                 int32_t* __restrict__ h, int8_t* __restrict__ wd,
                                                 unsigned long long* __restrict__ jbound) {
  __shared__ double red[2][4];
  const int mu = blockIdx.x, t = threadIdx.x;
  double m = 0.0, prop = 0.0;
  for (int64_t P = t; P < naux; P += 256) {
    const int e = b_exp[P * nao + mu];
    m = fmax(m, fabs(ldexp(rho[P], e)));
    prop += drho[P] * ldexp(1.0, e);
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    m = fmax(m, __shfl_xor(m, off));
    prop += __shfl_xor(prop, off);
  }
  if ((t & 63) == 0) {
    red[0][t >> 6] = m;
    red[1][t >> 6] = prop;
  }
  __syncthreads();
  m = fmax(fmax(red[0][0], red[0][1]), fmax(red[0][2], red[0][3]));
  const int e = exp_of_max(m);
  if (t == 0) {
    h[mu] = e;
    const double pr = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
    const double bnd = (double)naux * ldexp(1.0, e) * kap_j + pr;
    atomicMax(jbound, (unsigned long long)__double_as_longlong(bnd));
  }
  const int64_t plane = (int64_t)nao * naux_pad;
  int8_t* dst = wd + (int64_t)mu * naux_pad;
  for (int64_t P = t; P < naux_pad; P += 256) {
    uint64_t wv = 0;
    if (P < naux) wv = digit_word(ldexp(rho[P], b_exp[P * nao + mu]), e);
    for (int a = 0; a < S; ++a) dst[a * plane + P] = (int8_t)digit_byte(wv, a + 1);
  }
}

// 4 x 4 byte transpose: byte p of t[c] = byte c of v[p].
__device__ __forceinline__ void transpose4(uint32_t v0, uint32_t v1, uint32_t v2, uint32_t v3,
                                           uint32_t& t0, uint32_t& t1, uint32_t& t2,
                                           uint32_t& t3) {
  // __builtin_amdgcn_perm(hi, lo, sel): byte i of the result is byte sel_i of
  // the 64-bit value (hi << 32) | lo.
  const uint32_t lo01 = __builtin_amdgcn_perm(v1, v0, 0x05010400u);  // v0b0 v1b0 v0b1 v1b1
  const uint32_t hi01 = __builtin_amdgcn_perm(v1, v0, 0x07030602u);  // v0b2 v1b2 v0b3 v1b3
  const uint32_t lo23 = __builtin_amdgcn_perm(v3, v2, 0x05010400u);
  const uint32_t hi23 = __builtin_amdgcn_perm(v3, v2, 0x07030602u);
  t0 = __builtin_amdgcn_perm(lo23, lo01, 0x05040100u);
  t1 = __builtin_amdgcn_perm(lo23, lo01, 0x07060302u);
  t2 = __builtin_amdgcn_perm(hi23, hi01, 0x05040100u);
  t3 = __builtin_amdgcn_perm(hi23, hi01, 0x07060302u);
}

// Integer sums of J over one split of the aux range, for row mu and nu <= mu:
//   Sj[g][mu][nu] += sum_P sum_{a+b=g} wd[a][mu][P] Bd[b][P, mu][nu]  (int64 atomics)
// Thread (pl, c) owns the 16 nu of chunk c and the groups of 4 consecutive P
// congruent to pl; the four B rows of a group are transposed in registers so
// that v_dot4 runs over P; partial sums are combined over pl in LDS.
template <int S>
__global__ __launch_bounds__(256) void k_j_dig(const int8_t* __restrict__ Bd, int64_t bplane,
                                               int ldk, const int8_t* __restrict__ wd,
                                               int naux_pad, int64_t naux, int nao, int nsplit,
                                               unsigned long long* __restrict__ Sj) {
  __shared__ int red[256 * 17];
  const int mu = blockIdx.x, split = blockIdx.y, t = threadIdx.x;
  const int64_t ngrp = (naux + 3) / 4;
  const int64_t g_lo = split * ngrp / nsplit, g_hi = (split + 1) * ngrp / nsplit;
  const int nch = mu / 16 + 1;
  const int64_t wplane = (int64_t)nao * naux_pad;
  const int8_t* wrow = wd + (int64_t)mu * naux_pad;
  const int64_t nn = (int64_t)nao * nao;
  const int64_t prow = (int64_t)nao * ldk;
  for (int cbase = 0; cbase < nch; cbase += 256) {
    const int ncur = min(256, nch - cbase);
    const int npl = 256 / ncur;
    const int pl = t / ncur, c = cbase + (t - pl * ncur);
    int acc[S][16];
#pragma unroll
    for (int g = 0; g < S; ++g)
#pragma unroll
      for (int j = 0; j < 16; ++j) acc[g][j] = 0;
    if (pl < npl) {
      const int8_t* bbase = Bd + (int64_t)mu * ldk + c * 16;
      for (int64_t G = g_lo + pl; G < g_hi; G += npl) {
        const int64_t P0 = 4 * G;
        int wv[S];
#pragma unroll
        for (int a = 0; a < S; ++a) wv[a] = *reinterpret_cast<const int*>(wrow + a * wplane + P0);
#pragma unroll
        for (int b = 0; b < S; ++b) {
          i32x4 v[4];
#pragma unroll
          for (int p = 0; p < 4; ++p)
            v[p] = P0 + p < naux
                       ? *reinterpret_cast<const i32x4*>(bbase + b * bplane + (P0 + p) * prow)
                       : i32x4{0, 0, 0, 0};
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            uint32_t tt[4];
            transpose4((uint32_t)v[0][j], (uint32_t)v[1][j], (uint32_t)v[2][j], (uint32_t)v[3][j],
                       tt[0], tt[1], tt[2], tt[3]);
#pragma unroll
            for (int a = 0; a < S - b; ++a)
#pragma unroll
              for (int cc = 0; cc < 4; ++cc)
                acc[a + b][4 * j + cc] =
                    __builtin_amdgcn_sdot4(wv[a], (int)tt[cc], acc[a + b][4 * j + cc], false);
          }
        }
      }
    }
#pragma unroll
    for (int g = 0; g < S; ++g) {
      __syncthreads();
#pragma unroll
      for (int j = 0; j < 16; ++j) red[t * 17 + j] = acc[g][j];
      __syncthreads();
      for (int item = t; item < ncur * 16; item += 256) {
        const int cc = item >> 4, j = item & 15;
        int sum = 0;
        for (int p = 0; p < npl; ++p) sum += red[(p * ncur + cc) * 17 + j];
        const int nu = (cbase + cc) * 16 + j;
        if (nu <= mu)
          atomicAdd(&Sj[g * nn + (int64_t)mu * nao + nu], (unsigned long long)(long long)sum);
      }
    }
  }
}

// J[mu][nu] = J[nu][mu] = sum_{g = s+1 .. 2} ldexp(Sj[g], h_mu + 4 - 8 g), nu <= mu.
__global__ void k_j_recombine(const unsigned long long* __restrict__ Sj, int S, int nao,
                              const int32_t* __restrict__ h, double* __restrict__ J) {
  const int64_t nn = (int64_t)nao * nao;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nn;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int mu = (int)(e / nao), nu = (int)(e - (int64_t)mu * nao);
    if (nu > mu) continue;
    double z = 0.0;
    for (int g = S + 1; g >= 2; --g)
      z += ldexp((double)(long long)Sj[(int64_t)(g - 2) * nn + e], h[mu] + 4 - 8 * g);
    J[e] = z;
    J[(int64_t)nu * nao + mu] = z;
  }
}

inline unsigned cap(int64_t n, int64_t c = 65536) {
  int64_t g = (n + 255) / 256;
  return (unsigned)(g < 1 ? 1 : (g > c ? c : g));
}

template <int S>
hipError_t x_dig_s(hipStream_t st, const int8_t* Bd, int64_t bplane, int64_t M, int ldk,
                   const int32_t* b_exp, const int8_t* dC, int ncp, const int32_t* f_col,
                   int nocc, double* X, unsigned long long* xmax, int nao, int pblk,
                   const int8_t* Dd, const int32_t* d_exp, double* rowdot) {
  const unsigned gx = (unsigned)((M + 63) / 64);
#define DFJK_XD(NFW, NH)                                                                        \
  do {                                                                                          \
    constexpr int NT_ = 16 * (NFW) * (NH);                                                      \
    hipLaunchKernelGGL((k_x_dig<S, NFW, NH>), dim3(gx * (unsigned)(ncp / NT_)),                 \
                       dim3(256 * (NH)), 0, st, Bd, bplane, M, ldk, b_exp, dC, ncp, f_col, nocc, \
                       X, xmax, nao, pblk, Dd, d_exp, rowdot);                                  \
  } while (0)
  if (ncp % 96 == 0) {
    if constexpr (S <= 2) DFJK_XD(6, 1);
    else DFJK_XD(3, 2);
  } else if (ncp % 64 == 0) {
    if constexpr (S <= 3) DFJK_XD(4, 1);
    else DFJK_XD(2, 2);
  } else {
    DFJK_XD(1, 2);
  }
#undef DFJK_XD
  return hipGetLastError();
}

}  // namespace

hipError_t launch_slice_planes(hipStream_t st, const double* A, int64_t rows, int cols, int ldk,
                               const int32_t* e, int planes, int8_t* dig, int packed) {
  if (rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_slice_planes, dim3(cap(rows * (ldk / 16))), dim3(256), 0, st, A, rows, cols,
                     ldk, e, planes, dig, packed);
  return hipGetLastError();
}

hipError_t launch_x_dig(hipStream_t st, int s, const int8_t* Bd, int64_t bplane, int64_t naux,
                        int nao, int ldk, const int32_t* b_exp, const int8_t* dC, int ncp,
                        const int32_t* f_col, int nocc, double* X, unsigned long long* xmax,
                        int pblk, const int8_t* Dd, const int32_t* d_exp, double* rowdot) {
  const int64_t M = naux * nao;
#define DFJK_XDS(SS) \
  return x_dig_s<SS>(st, Bd, bplane, M, ldk, b_exp, dC, ncp, f_col, nocc, X, xmax, nao, pblk, Dd, d_exp, rowdot)
  switch (s) {
    case 1: DFJK_XDS(1);
    case 2: DFJK_XDS(2);
    case 3: DFJK_XDS(3);
    case 4: DFJK_XDS(4);
    case 5: DFJK_XDS(5);
    case 6: DFJK_XDS(6);
    case 7: DFJK_XDS(7);
    case 8: DFJK_XDS(8);
    default: return hipErrorInvalidValue;
  }
#undef DFJK_XDS
}

hipError_t launch_rho_seq(hipStream_t st, const double* rowdot, const int32_t* b_exp,
                          const int32_t* d_exp, int64_t naux, int nao, double kap_row,
                          double kap_sum, double* rho, double* drho) {
  hipLaunchKernelGGL(k_rho_seq, dim3((unsigned)((naux + 63) / 64)), dim3(256), 0, st, rowdot,
                     b_exp, d_exp, naux, nao, kap_row, kap_sum, rho, drho);
  return hipGetLastError();
}

hipError_t launch_j_dig(hipStream_t st, int s, const int8_t* Bd, int64_t bplane, int ldk,
                        const double* rho, const double* drho, const int32_t* b_exp, int64_t naux,
                        int nao, int naux_pad, int nsplit, double kap_j, int32_t* h, int8_t* wd,
                        unsigned long long* Sj, unsigned long long* jbound, double* J) {
  const int64_t nn = (int64_t)nao * nao;
  hipError_t e = launch_fill_u64(st, Sj, (int64_t)s * nn, 0ull);
  if (e != hipSuccess) return e;
  e = launch_fill_u64(st, jbound, 1, 0ull);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_slice_w, dim3((unsigned)nao), dim3(256), 0, st, rho, drho, b_exp, naux, nao,
                     s, naux_pad, kap_j, h, wd, jbound);
  const dim3 grid((unsigned)nao, (unsigned)nsplit);
#define DFJK_JD(SS)                                                                            \
  hipLaunchKernelGGL((k_j_dig<SS>), grid, dim3(256), 0, st, Bd, bplane, ldk, wd, naux_pad, naux, \
                     nao, nsplit, Sj)
  switch (s) {
    case 1: DFJK_JD(1); break;
    case 2: DFJK_JD(2); break;
    case 3: DFJK_JD(3); break;
    case 4: DFJK_JD(4); break;
    case 5: DFJK_JD(5); break;
    case 6: DFJK_JD(6); break;
    case 7: DFJK_JD(7); break;
    case 8: DFJK_JD(8); break;
    default: return hipErrorInvalidValue;
  }
#undef DFJK_JD
  hipLaunchKernelGGL(k_j_recombine, dim3(cap(nn, 4096)), dim3(256), 0, st, Sj, s, nao, h, J);
  return hipGetLastError();
}

}  // namespace dfjk
