// INT8-slice emulation of the two FP64 products of the exchange build
// (Sec. 3.2; Eqs. 5-6 blocked as Eqs. df-k-blk-1/2 of Sec. 3.3) on gfx950
// v_mfma_i32_16x16x64_i8.
//
//   X product (Eq. 5): rows (P, mu) of B over nu  x  columns i of C over nu.
//   K product (Eq. 6): per aux block b, rows mu of X_b over (P in b, i), a
//                      symmetric rank-k update computed on lower 64x64 tiles.
//
// Every kept digit pair (a + b <= s + 1) is multiplied on the matrix cores and
// summed exactly in one int32 accumulator per anti-diagonal g = a + b; the
// accumulators are recombined in FP64, smallest weight first.
//
// MFMA operand layout (checked on gfx950): lane l holds row/column (l & 15)
// and 16 consecutive k "slots" of lane group (l >> 4); the result register r
// of lane l is row 4 (l >> 4) + r, column (l & 15).  The two operands of one
// product only have to agree on which k sits in which slot.
#include "dfjk_internal.h"

namespace dfjk {
namespace {

// 16 bytes per lane from a buffer resource (byte offset voff + soff) straight
// into LDS: lane i of the wave writes bytes 16 i .. 16 i + 15 after the
// wave-uniform LDS address lds_dst.  Completion is counted by vmcnt.
__device__ __forceinline__ void copy16_to_lds(__amdgpu_buffer_rsrc_t r, void* lds_dst, int voff,
                                              int soff) {
  __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (__attribute__((address_space(3))) void*)lds_dst, 16,
                                           voff, soff, 0, 0);
}

// 4 x 4 byte transpose of d[0..3] with byte permutes: t[b] holds byte b of
// d[0], d[1], d[2], d[3] in its bytes 0..3.  (v_perm_b32: selector values 0-3
// take bytes of the second operand, 4-7 bytes of the first.)
__device__ __forceinline__ void transpose4x4(const uint32_t d[4], uint32_t t[4]) {
  const uint32_t p01 = __builtin_amdgcn_perm(d[1], d[0], 0x05010400u);  // d0b0 d1b0 d0b1 d1b1
  const uint32_t q01 = __builtin_amdgcn_perm(d[1], d[0], 0x07030602u);  // d0b2 d1b2 d0b3 d1b3
  const uint32_t p23 = __builtin_amdgcn_perm(d[3], d[2], 0x05010400u);
  const uint32_t q23 = __builtin_amdgcn_perm(d[3], d[2], 0x07030602u);
  t[0] = __builtin_amdgcn_perm(p23, p01, 0x05040100u);
  t[1] = __builtin_amdgcn_perm(p23, p01, 0x07060302u);
  t[2] = __builtin_amdgcn_perm(q23, q01, 0x05040100u);
  t[3] = __builtin_amdgcn_perm(q23, q01, 0x07060302u);
}

// Digits 1..S of eight values (one exponent e) as S rows of 8 bytes: row a
// (0-based) holds digit a + 1 of v[j] in its byte j, i.e. byte 7 - a of the
// digit word of v[j], formed by byte transposes of the offset words and one
// flip of the offset per packed word (digit 1 carries no offset).
template <int S>
__device__ __forceinline__ void digit_rows8(const double* v, int e, uint2* out) {
  uint32_t tr[2][2][4];  // [half of the 8 values][low / high 32 bits][byte]
#pragma unroll
  for (int g = 0; g < 2; ++g) {
    uint32_t lo[4], hi[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint64_t w = digit_word_offset(v[4 * g + j], e);
      lo[j] = (uint32_t)w;
      hi[j] = (uint32_t)(w >> 32);
    }
    transpose4x4(lo, tr[g][0]);
    transpose4x4(hi, tr[g][1]);
  }
  // digit k (1 = most significant) is byte 8 - k of the word
#pragma unroll
  for (int a = 0; a < S; ++a) {
    const int byte = 7 - a;
    const uint32_t flip = a == 0 ? 0u : 0x80808080u;
    out[a] = make_uint2(tr[0][byte >> 2][byte & 3] ^ flip, tr[1][byte >> 2][byte & 3] ^ flip);
  }
}

// ---------------------------------------------------------------------------
// X = B C.  Workgroup: 8 waves, tile 64 rows (P, mu) x 16*NF columns i.  For
// the MFMAs, waves w and w + 4 own rows 16 (w % 4) .. + 15 and split the
// columns in halves.  For loading and slicing, wave w takes rows 8 w .. 8 w + 7
// of the tile, eight lanes per row: lane m = l & 7 of a row reads k = 16 j +
// 2 m + {0, 1} (j = 0..3) of each 64-wide sub-chunk, so that every load
// instruction covers whole 128-byte lines, slices its 8 values in registers
// and writes their digits as 8 consecutive bytes of the LDS A row: MFMA slot
// 8 (m & 1) + 2 j + h of lane group m >> 1 holds k = 16 j + 2 m + h (the C
// digit planes are stored in the same order).  The C digits of the chunk are
// staged in LDS as well.  The next chunk of B (and D) is prefetched into
// registers while the current one is multiplied.  Optionally the row dots
// sum_nu B[P][mu][nu] D[mu][nu] (rho, Eq. 3) are formed from the same B values.
// X layout 0: X[row][i]; layout 1 (blocked): X_b rows, element
// ((b nao + mu) pblk + P - P0) nocc + i.
// ---------------------------------------------------------------------------
//
// Packed B (PK): B_P stored as its lower triangle, row mu >= nu, element
// (mu, nu) at mu (mu + 1) / 2 + nu (B_P is symmetric).  A tile (P, rows
// mu0 .. mu0 + 63) reads each 64-wide nu chunk c of its rows in one of three
// ways: below the tile's diagonal block the rows of the triangle (contiguous,
// the same lane layout as dense B); the diagonal block element by element
// (mu >= nu from the row, mu < nu from the mirror); above it the mirrored block,
// stored as rows nu of the triangle over the tile's mu: then wave w takes the
// eight nu that lane-in-row w would take and lane l takes tile row l, so every
// load instruction reads 64 consecutive mu of one stored row (512 B), and the
// digits are written to LDS row l in the same slots.  Each element is sliced
// with the exponent of the row it is used for (that of mu in both
// orientations), so the result is bit-identical to dense B.  The tiles of one
// P are handed to one XCD together, and tile t visits chunk (s - t) mod n at
// step s: the two tiles that read one stored block (one directly, one
// mirrored) read it at the same step, so the second read is served by L2.
//
// E extra anti-diagonals (0 or 1): the pairs a + b <= s + 1 + E (a, b <= s)
// are formed, S + E int32 accumulators per output.
//
// At s <= 3 the packed-B kernel is held to 128 VGPRs (two workgroups per CU;
// a few spilled words), which measured faster than 150 VGPRs at one.
template <int S, int NF, bool FULLK, int KSUB, bool PK, int E>
__global__ __launch_bounds__(512)
__attribute__((amdgpu_waves_per_eu((PK && S <= 3 && KSUB == 1 && NF <= 8) ? 4 : 1))) void k_x_int8(
    const double* __restrict__ B, int64_t M, int K, const int32_t* __restrict__ b_exp,
    const int8_t* __restrict__ dC, int ncp, int kp, const int32_t* __restrict__ f_col, int nocc,
    double* __restrict__ X, int xlayout, unsigned long long* __restrict__ xmax, int nao, int pblk,
    const double* __restrict__ D, double* __restrict__ rowdot,
    const unsigned long long* __restrict__ cmask, int32_t* __restrict__ dbg) {
  constexpr int NT = 16 * NF, NFW = NF / 2;
  constexpr int KC = 64 * KSUB, ROW = KC;  // LDS rows: KC k bytes, units swizzled per 64 B
  constexpr int CUNITS = S * NT * 4 * KSUB;     // 16-byte units of C digits per chunk
  constexpr int CPER = (CUNITS + 511) / 512;
  constexpr int NV = 8 * KSUB;                  // B values sliced per lane per chunk
  // Two LDS stages when they fit (KSUB == 1): the digits of chunk c + 1 are
  // written while chunk c is multiplied, one barrier per chunk.
  constexpr int NBUF = (KSUB == 1 && 2 * S * (64 + NT) * ROW + 1024 <= 160 * 1024) ? 2 : 1;
  __shared__ __attribute__((aligned(16))) int8_t As[NBUF][S][64][ROW];
  // The two C stages are separate arrays, so that the compiler can tell the
  // stage being copied into from the one being read.  With two stages each
  // has 16 spare rows (1 KB) at its end: the landing block of the copies of
  // waves that have no block left in a chunk (every wave issues the same
  // number of copies; never read).
  constexpr int CPAD = NBUF == 2 && CUNITS % 512 ? 16 : 0;
  __shared__ __attribute__((aligned(16))) int8_t Cs0[S * NT + CPAD][ROW];
  __shared__ __attribute__((aligned(16))) int8_t Cs1[NBUF == 2 ? S * NT + CPAD : 1][ROW];
#define DFJK_CSB(BUF) ((BUF) ? Cs1 : Cs0)
  // (+ 8 bytes: the chunk mask of tile_chunks)
  static_assert(sizeof(As) + sizeof(Cs0) + sizeof(Cs1) + 8 <= kLdsLimit, "X tile exceeds LDS");

  const int t = threadIdx.x, w = t >> 6, l = t & 63, q = l >> 4, r16 = l & 15;
  const int wrow = w & 3, half = w >> 2;  // waves w and w + 4 share 16 rows
  const int lrow = 8 * w + (l >> 3), lm = l & 7;  // loader: tile row, lane within row
  // Workgroups that run together share the basis-row tile mu0..mu0+63 (and so
  // the same rows of D, which stay in L2) and differ in the aux index P.
  // With several column tiles (gridDim.y) the tiles are numbered (row tile,
  // column tile) and handed to the XCDs in contiguous ranges, so that the
  // column tiles of one row tile read its B rows from one L2.
  const int ncol = gridDim.y;
  int64_t rt = blockIdx.x;
  int ct = 0;
  if (ncol > 1) {
    const int64_t lid = xcd_order(blockIdx.x + (int64_t)blockIdx.y * gridDim.x,
                                  (int64_t)gridDim.x * ncol);
    rt = lid / ncol;
    ct = (int)(lid - rt * ncol);
  } else if (PK) {
    rt = xcd_order(blockIdx.x, gridDim.x);
  }
  int64_t m0 = rt * 64;
  int64_t ptile = 0;  // PK: the tile's aux index; mu0 its first row
  int mu0 = 0;
  if constexpr (PK) {
    const int nmt = (nao + 63) >> 6;
    ptile = rt / nmt;
    mu0 = (int)(rt - ptile * nmt) * 64;
    m0 = ptile * nao + mu0;
  } else if (nao % 64 == 0) {
    const int64_t naux = M / nao;
    const int64_t mt = rt / naux, P = rt - mt * naux;
    m0 = P * nao + mt * 64;
  }
  const int n0 = ct * NT;
  // Rows past M (PK: past nao) read an in-bounds row; their digits and sums
  // are discarded.
  const int64_t arow = m0 + lrow;
  const bool aok = PK ? mu0 + lrow < nao : arow < M;
  const double* brow = B + (aok && !PK ? arow : 0) * (int64_t)K + 2 * lm;
  const int e_a = aok ? b_exp[arow] : 0;
  const bool want_rd = D != nullptr;
  const double* drow = (want_rd ? D : B) + (aok ? (arow % nao) : 0) * (int64_t)K + 2 * lm;
  const int nch = (K + KC - 1) / KC;
  int8_t* adst = &As[0][0][lrow][swz(lrow, lm >> 1) + (lm & 1) * 8];
  // Screened B: only the KC-wide nu chunks that meet a kept block in some row
  // of this tile are visited (the rest of the tile is zero).
  const unsigned long long live = cmask ? tile_chunks<KSUB>(cmask, m0, M, nao, w, l) : 0ull;

  const int8_t* csrc[CPER];
  int cdst[CPER];
#pragma unroll
  for (int i = 0; i < CPER; ++i) {
    const int u = t + 512 * i;
    const int uu = u < CUNITS ? u : 0;
    const int per_plane = NT * 4 * KSUB;
    const int a = uu / per_plane, rem = uu - a * per_plane;
    const int col = rem / (4 * KSUB), part = rem - col * (4 * KSUB);
    // C digit planes tiled by 64-wide k chunks: (a, chunk c, column) rows of 64 B
    csrc[i] = dC + ((int64_t)(a * (kp >> 6) + (part >> 2)) * ncp + n0 + col) * 64 + (part & 3) * 16;
    cdst[i] = (a * NT + col) * ROW + (part >> 2) * 64 + swz(col, part & 3);
  }

  // With two LDS stages the C digits go straight from memory to LDS (one
  // 1 KB block of 16 columns of one plane per wave instruction; lane i lands
  // at byte 16 i of the block, so it fetches the unit that the row swizzle
  // puts there).
  // The copies are buffer loads (byte offsets from a resource over the S
  // digit planes of C, bounds-checked by the hardware).
  constexpr int CINS = CUNITS / 64, CIW = (CINS + 7) / 8;
  const __amdgpu_buffer_rsrc_t crsrc = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<int8_t*>(dC), (short)0, S * ncp * kp, 0x00020000);
  int coff[NBUF == 2 ? CIW : 1];
  // Two-stage full-K path: B and D rows are read by buffer loads too (byte
  // offsets from resources over this tile's 64 rows of B and of D, chunk
  // offset in a scalar), so no address registers are rewritten per chunk.
  const __amdgpu_buffer_rsrc_t brsrc = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<double*>(B + m0 * (int64_t)K), (short)0, 64 * K * 8, 0x00020000);
  const __amdgpu_buffer_rsrc_t drsrc = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<double*>((want_rd ? D : B) + (PK ? mu0 : m0 % nao) * (int64_t)K), (short)0,
      (PK ? min(64, nao - mu0) : 64) * K * 8, 0x00020000);
  const int vbo = (lrow * K + 2 * lm) * 8;
  // PK: a resource over the stored triangle of B_P, and the per-lane parts of
  // the offsets (rows clamped to nao - 1: padding rows read a real row).  The
  // mirrored loader's lane takes tile row l (exponent e_t, LDS row l).
  const int nao1 = nao - 1;
  const int mu_c = PK ? min(mu0 + lrow, nao1) : 0;
  const int muT = mu0 + l, muT_c = PK ? min(muT, nao1) : 0;
  const __amdgpu_buffer_rsrc_t bprsrc = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<double*>(B + (PK ? ptile * ((int64_t)nao * (nao + 1) / 2) : 0)), (short)0,
      PK ? (int)((int64_t)nao * (nao + 1) / 2 * 8) : 0, 0x00020000);
  const int voffL = (mu_c * (mu_c + 1) / 2 + 2 * lm) * 8;
  const int voffT = muT_c * 8;
  const int vboD = ((PK ? mu_c - mu0 : lrow) * K + 2 * lm) * 8;
  const int e_t = (PK && muT < nao) ? b_exp[ptile * nao + muT] : 0;
  int8_t* adstT = &As[0][0][l][swz(l, w >> 1) + (w & 1) * 8];
  const int wlm = __builtin_amdgcn_readfirstlane(w);  // the mirrored loader's lane-in-row
  if constexpr (NBUF == 2) {
#pragma unroll
    for (int j = 0; j < CIW; ++j) {
      const int ins = w + 8 * j;
      const int u0 = (ins < CINS ? ins : 0) * 64;
      const int a = u0 / (NT * 4 * KSUB), col0 = (u0 - a * NT * 4 * KSUB) / (4 * KSUB);
      const int col = col0 + (l >> 2), part = (l & 3) ^ ((col >> 1) & 3);
      coff[j] = ((a * (kp >> 6)) * ncp + n0 + col) * 64 + part * 16;
    }
  }

  constexpr int G = S + E;  // anti-diagonals kept
  i32x4 acc[G][NFW];
#pragma unroll
  for (int g = 0; g < G; ++g)
#pragma unroll
    for (int f = 0; f < NFW; ++f) acc[g][f] = i32x4{0, 0, 0, 0};
  double rd = 0.0;
  // Two-stage full-K path: B_P and D are symmetric, so the row dots of rho
  // need only the chunks up to the tile's diagonal block cdiag (its rows are
  // mu = 64 cdiag + lrow): chunks below it count twice, the diagonal block by
  // element (2 below the diagonal, 1 on it, 0 above; exact weights), chunks
  // past it not at all, and their D rows are not read.
  constexpr bool TRI = NBUF == 2 && FULLK;
  constexpr bool RDTRI = TRI || PK;  // row dots over the chunks up to the diagonal block
  const int cdiag = PK ? (mu0 >> 6) : (TRI ? (int)((m0 % nao) >> 6) : 0);

  double v[NV], dv[NV];
  i32x4 cpre[NBUF == 1 ? CPER : 1];
#define DFJK_X_LOAD(CC)                                                                    \
  {                                                                                        \
    const int kb0 = (CC) * KC;                                                             \
    if constexpr (PK) {                                                                    \
      if ((CC) < cdiag) { /* rows of the triangle: 4 loads of 16 B */                      \
        _Pragma("unroll") for (int j = 0; j < 4; ++j) {                                    \
          const double2 pb = __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128( \
              bprsrc, voffL + 128 * j, kb0 * 8, 0));                                       \
          v[2 * j] = pb.x;                                                                 \
          v[2 * j + 1] = pb.y;                                                             \
        }                                                                                  \
      } else if ((CC) == cdiag) { /* diagonal block: element by element (columns past */  \
        /* nao read column nao - 1 and are zeroed when staged, so that no load waits) */   \
        _Pragma("unroll") for (int j = 0; j < 8; ++j) {                                    \
          const int nu = kb0 + 16 * (j >> 1) + 2 * lm + (j & 1);                           \
          const int nuc = min(nu, nao1);                                                   \
          const int off = nuc <= mu_c ? mu_c * (mu_c + 1) / 2 + nuc : nuc * (nuc + 1) / 2 + mu_c; \
          v[j] = __builtin_bit_cast(double,                                                \
              __builtin_amdgcn_raw_buffer_load_b64(bprsrc, off * 8, 0, 0));                \
        }                                                                                  \
      } else { /* mirrored block: stored rows nu, 64 consecutive mu per load */            \
        _Pragma("unroll") for (int j = 0; j < 8; ++j) {                                    \
          const int nu = kb0 + 16 * (j >> 1) + 2 * wlm + (j & 1);                           \
          const int nuc = min(nu, nao1);                                                   \
          v[j] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(          \
              bprsrc, voffT, nuc * (nuc + 1) / 2 * 8, 0));                                 \
        }                                                                                  \
      }                                                                                    \
      if (want_rd && (CC) <= cdiag) {                                                      \
        _Pragma("unroll") for (int j = 0; j < 4; ++j) {                                    \
          const double2 pd = __builtin_bit_cast(                                           \
              double2, __builtin_amdgcn_raw_buffer_load_b128(drsrc, vboD + 128 * j, kb0 * 8, 0)); \
          dv[2 * j] = pd.x;                                                                \
          dv[2 * j + 1] = pd.y;                                                            \
        }                                                                                  \
      }                                                                                    \
    } else if constexpr (TRI) {                                                            \
      _Pragma("unroll") for (int j = 0; j < 4; ++j) {                                      \
        const double2 pb = __builtin_bit_cast(                                             \
            double2, __builtin_amdgcn_raw_buffer_load_b128(brsrc, vbo + 128 * j, kb0 * 8, 0)); \
        v[2 * j] = pb.x;                                                                   \
        v[2 * j + 1] = pb.y;                                                               \
      }                                                                                    \
      if (want_rd && (CC) <= cdiag) {                                                      \
        _Pragma("unroll") for (int j = 0; j < 4; ++j) {                                    \
          const double2 pd = __builtin_bit_cast(                                           \
              double2, __builtin_amdgcn_raw_buffer_load_b128(drsrc, vbo + 128 * j, kb0 * 8, 0)); \
          dv[2 * j] = pd.x;                                                                \
          dv[2 * j + 1] = pd.y;                                                            \
        }                                                                                  \
      }                                                                                    \
    } else if (FULLK) {                                                                    \
      _Pragma("unroll") for (int j = 0; j < NV / 2; ++j) {                                 \
        const int off = kb0 + 64 * (j >> 2) + 16 * (j & 3);                                \
        const double2 p = *reinterpret_cast<const double2*>(brow + off);                   \
        v[2 * j] = p.x;                                                                    \
        v[2 * j + 1] = p.y;                                                                \
      }                                                                                    \
      /* D rows are read even when unused (drow then points into B), so that */           \
      /* every step issues the same number of loads */                                      \
      _Pragma("unroll") for (int j = 0; j < NV / 2; ++j) {                                 \
        const int off = kb0 + 64 * (j >> 2) + 16 * (j & 3);                                \
        const double2 p = *reinterpret_cast<const double2*>(drow + off);                   \
        dv[2 * j] = p.x;                                                                   \
        dv[2 * j + 1] = p.y;                                                               \
      }                                                                                    \
    } else {                                                                               \
      _Pragma("unroll") for (int j = 0; j < NV; ++j) {                                     \
        const int off = kb0 + 64 * (j >> 3) + 16 * ((j >> 1) & 3) + (j & 1);              \
        const int kk = off + 2 * lm;                                                       \
        v[j] = kk < K ? brow[off] : 0.0;                                                   \
        dv[j] = (want_rd && kk < K) ? drow[off] : 0.0;                                     \
      }                                                                                    \
    }                                                                                      \
    if constexpr (NBUF == 1) {                                                             \
      _Pragma("unroll") for (int i = 0; i < CPER; ++i) {                                   \
        if (t + 512 * i < CUNITS)                                                          \
          cpre[i] = *reinterpret_cast<const i32x4*>(csrc[i] + (int64_t)(kb0 >> 6) * ncp * 64); \
      }                                                                                    \
    }                                                                                      \
  }
  // C digits of chunk CC straight into LDS stage BUF (two-stage loop only).
  // A wave with no block left in the last round skips it (wave-uniform; the
  // barrier's count concerns only the loads issued after the copies).
  const int wcu = __builtin_amdgcn_readfirstlane(w);
#define DFJK_X_CDMA(BUF, CC)                                                                \
  _Pragma("unroll") for (int j = 0; j < CIW; ++j) {                                        \
    const int ins = wcu + 8 * j;                                                           \
    /* block ins: plane a, columns col0 .. col0 + 15 */                                    \
    if (j + 1 < CIW || ins < CINS) {                                                       \
      int8_t* dst = &DFJK_CSB(BUF)[(ins * 64) / 4][0];                                      \
      copy16_to_lds(crsrc, dst, coff[j], (CC) * ncp * 64);                                 \
    }                                                                                      \
  }

  // Digits of chunk CC, whose B values and C digits sit in registers, into
  // LDS stage BUF (and its B.D row-dot terms into rd / rd_off).
#define DFJK_X_STAGE(BUF, CC)                                                                   \
  {                                                                                             \
    if (PK && (nao & 63) && (CC) >= cdiag) { /* PK: columns past nao are zero */                \
      _Pragma("unroll") for (int j = 0; j < 8; ++j) {                                           \
        const int nu = (CC) * 64 + 16 * (j >> 1) + 2 * ((CC) == cdiag ? lm : wlm) + (j & 1);    \
        if (nu >= nao) v[j] = 0.0;                                                              \
      }                                                                                         \
    }                                                                                           \
    /* row-dot terms (zeroed after the loop when there is no D) */                              \
    if constexpr (RDTRI) {                                                                      \
      /* below the diagonal block a uniform doubling (v + v == 2 v exactly); at */              \
      /* s <= 3 the single weighted form, which keeps two workgroups per CU */                  \
      if (S >= 4 && (CC) < cdiag) {                                                             \
        _Pragma("unroll") for (int j = 0; j < NV; ++j) rd = fma(v[j] + v[j], dv[j], rd);        \
      } else if (S >= 4 ? (CC) == cdiag : (CC) <= cdiag) {                                      \
        _Pragma("unroll") for (int j = 0; j < NV; ++j) {                                        \
          const int kr = 16 * (j >> 1) + 2 * lm + (j & 1) + 64 * ((CC) - cdiag); /* k - mu0 */  \
          const double wgt = kr < lrow ? 2.0 : (kr == lrow ? 1.0 : 0.0);                        \
          rd = fma(v[j] * wgt, dv[j], rd);                                                      \
        }                                                                                       \
      }                                                                                         \
    } else {                                                                                    \
      _Pragma("unroll") for (int j = 0; j < NV; ++j) rd = fma(v[j], dv[j], rd);                 \
    }                                                                                           \
    if (PK && (CC) > cdiag) { /* mirrored block: this lane's values are tile row l's */         \
      uint2 rows[S];                                                                            \
      digit_rows8<S>(v, e_t, rows);                                                             \
      _Pragma("unroll") for (int a = 0; a < S; ++a)                                             \
        *reinterpret_cast<uint2*>(adstT + ((BUF) * S + a) * 64 * ROW) = rows[a];                \
    } else {                                                                                    \
      _Pragma("unroll") for (int sub = 0; sub < KSUB; ++sub) {                                  \
        uint2 rows[S];                                                                          \
        digit_rows8<S>(&v[8 * sub], e_a, rows);                                                 \
        _Pragma("unroll") for (int a = 0; a < S; ++a)                                           \
          *reinterpret_cast<uint2*>(adst + ((BUF) * S + a) * 64 * ROW + sub * 64) = rows[a];    \
      }                                                                                         \
    }                                                                                           \
    if constexpr (NBUF == 1) {                                                                  \
      _Pragma("unroll") for (int i = 0; i < CPER; ++i) {                                        \
        if (t + 512 * i < CUNITS)                                                               \
          *reinterpret_cast<i32x4*>(&DFJK_CSB(BUF)[0][0] + cdst[i]) = cpre[i];                  \
      }                                                                                         \
    }                                                                                           \
  }
  // MFMAs of the chunk held in LDS stage BUF.
#define DFJK_X_MMA(BUF)                                                                         \
  _Pragma("unroll") for (int sub = 0; sub < KSUB; ++sub) {                                      \
    i32x4 af[S];                                                                                \
    _Pragma("unroll") for (int a = 0; a < S; ++a) af[a] = *reinterpret_cast<const i32x4*>(      \
        &As[BUF][a][wrow * 16 + r16][sub * 64 + swz(wrow * 16 + r16, q)]);                      \
    _Pragma("unroll") for (int f = 0; f < NFW; ++f) {                                           \
      const int col = (half * NFW + f) * 16 + r16;                                              \
      i32x4 bf[S];                                                                              \
      _Pragma("unroll") for (int b = 0; b < S; ++b) bf[b] =                                     \
          *reinterpret_cast<const i32x4*>(&DFJK_CSB(BUF)[b * NT + col][sub * 64 + swz(col, q)]); \
      _Pragma("unroll") for (int a = 0; a < S; ++a)                                             \
        _Pragma("unroll") for (int b = 0; b < (S - a + E < S ? S - a + E : S); ++b)             \
          acc[a + b][f] =                                                                       \
            __builtin_amdgcn_mfma_i32_16x16x64_i8(af[a], bf[b], acc[a + b][f], 0, 0, 0);        \
    }                                                                                           \
  }

  // PK: tile mt visits chunk (step - mt) mod nch at each step (all nch chunks,
  // wrapping around); otherwise ascending (screened: the live chunks only).
  const int cfirst = PK ? (nch - cdiag % nch) % nch : 0;
  const int clast = PK ? (cfirst + nch - 1) % nch : nch - 1;
  int c = cmask ? first_bit(live) : (nch > 0 ? cfirst : -1);
  auto next_of = [&](int cc) {
    if (cc < 0) return -1;
    if (cmask) return next_bit(live, cc);
    if (PK) return cc == clast ? -1 : (cc + 1 == nch ? 0 : cc + 1);
    return cc + 1 < nch ? cc + 1 : -1;
  };
  if constexpr (NBUF == 2) {
    // stage c into LDS 0, prefetch the next chunk into registers; then per
    // chunk: stage the next chunk into the other LDS buffer, prefetch the
    // one after, multiply the current one, one barrier.
    int cn = next_of(c);
    if (c >= 0) {
      DFJK_X_CDMA(0, c)
      DFJK_X_LOAD(c)
      DFJK_X_STAGE(0, c)
    }
    if (cn >= 0) DFJK_X_LOAD(cn)
    __builtin_amdgcn_s_waitcnt(0);  // this wave's C digits have landed in LDS
    __syncthreads();
    // One step with chunk c in stage BB: stage chunk cn's A digits into the
    // other stage, start the copy of chunk cn's C digits into the other stage,
    // issue the loads of chunk cnn (after the copies, in this order), multiply
    // chunk c and meet at the barrier.  Full K: the barrier is written out
    // (s_waitcnt + s_barrier, a compiler memory barrier) and waits only for
    // this wave's copies and LDS stores: the loads of chunk cnn, the only
    // vector-memory operations issued after the copies (8, or 4 when chunk cnn
    // is past the diagonal block and its D rows are not read), stay in flight
    // into the next step.  Ragged K: a workgroup barrier (waits for everything).
    static_assert(NV == 8, "two-stage X loop assumes 8 values per lane and chunk");
#define DFJK_X_STEP(BB)                                                                         \
  {                                                                                             \
    const int cnn = next_of(cn);                                                                \
    if (cn >= 0) DFJK_X_STAGE(1 - (BB), cn)                                                     \
    __builtin_amdgcn_sched_barrier(0);                                                          \
    if (cn >= 0) DFJK_X_CDMA(1 - (BB), cn)                                                      \
    __builtin_amdgcn_sched_barrier(0);                                                          \
    if (cnn >= 0) DFJK_X_LOAD(cnn)                                                              \
    __builtin_amdgcn_sched_barrier(0);                                                          \
    DFJK_X_MMA(BB)                                                                              \
    /* PK: chunk cnn's loads are 4 (rows), 8 (diagonal, mirrored) B loads, plus */              \
    /* 4 D loads up to the diagonal block */                                                    \
    if (PK && cnn >= 0 && cnn == cdiag && want_rd)                                              \
      asm volatile("s_waitcnt vmcnt(12) lgkmcnt(0)\n\ts_barrier" ::: "memory");                \
    else if (PK && cnn >= 0 && (cnn == cdiag || cnn > cdiag || want_rd))                       \
      asm volatile("s_waitcnt vmcnt(8) lgkmcnt(0)\n\ts_barrier" ::: "memory");                 \
    else if (PK && cnn >= 0)                                                                    \
      asm volatile("s_waitcnt vmcnt(4) lgkmcnt(0)\n\ts_barrier" ::: "memory");                 \
    else if (FULLK && cnn >= 0 && want_rd && cnn <= cdiag)                                      \
      asm volatile("s_waitcnt vmcnt(8) lgkmcnt(0)\n\ts_barrier" ::: "memory");                 \
    else if (FULLK && cnn >= 0)                                                                 \
      asm volatile("s_waitcnt vmcnt(4) lgkmcnt(0)\n\ts_barrier" ::: "memory");                 \
    else                                                                                        \
      __syncthreads();                                                                          \
    c = cn;                                                                                     \
    cn = cnn;                                                                                   \
  }
    while (c >= 0) {
      DFJK_X_STEP(0)
      if (c < 0) break;
      DFJK_X_STEP(1)
    }
#undef DFJK_X_STEP
  } else {
    if (c >= 0) DFJK_X_LOAD(c)
    while (c >= 0) {
      const int cn = next_of(c);
      __syncthreads();  // the previous chunk's LDS reads are done
      DFJK_X_STAGE(0, c)
      __syncthreads();  // A and C digits of chunk c are in LDS
      if (cn >= 0) DFJK_X_LOAD(cn)
      DFJK_X_MMA(0)
      c = cn;
    }
  }
  if (!want_rd) rd = 0.0;
#undef DFJK_X_MMA
#undef DFJK_X_STAGE
#undef DFJK_X_CDMA
#undef DFJK_X_LOAD
#undef DFJK_CSB

  if (rowdot) {
    // row dot = sum over the eight lanes of the row, fixed order
    rd += __shfl_xor(rd, 1);
    rd += __shfl_xor(rd, 2);
    rd += __shfl_xor(rd, 4);
    if (lm == 0 && aok && ct == 0) rowdot[arow] = rd;
  }

  // Recombination, X store, and the per-(block, mu) running max of |X|.
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int64_t row = m0 + wrow * 16 + q * 4 + r;
    const bool vr = PK ? mu0 + wrow * 16 + q * 4 + r < nao : row < M;
    const int er = vr ? b_exp[row] : 0;
    const int64_t P = PK ? ptile : (vr ? row / nao : 0);
    const int mu = (int)(row - P * nao);
    const int64_t b = P / pblk;
    double* xrow = xlayout ? X + (((b * nao + mu) * pblk + (P - b * pblk)) * (int64_t)nocc)
                           : X + row * (int64_t)nocc;
    double rmax = 0.0;
#pragma unroll
    for (int f = 0; f < NFW; ++f) {
      const int col = n0 + (half * NFW + f) * 16 + r16;
      if (vr && col < nocc) {
        const int base = er + f_col[col] + 4;
        double z = 0.0;
#pragma unroll
        for (int g = G + 1; g >= 2; --g) z += ldexp((double)acc[g - 2][f][r], base - 8 * g);
        xrow[col] = z;
        rmax = fmax(rmax, fabs(z));
        if (dbg) {  // test export: the int32 anti-diagonal sums of this tile
#pragma unroll
          for (int g = 0; g < G; ++g) dbg[((int64_t)g * M + row) * nocc + col] = acc[g][f][r];
        }
      }
    }
#pragma unroll
    for (int off = 1; off < 16; off <<= 1) rmax = fmax(rmax, __shfl_xor(rmax, off));
    if (r16 == 0 && vr)
      atomicMax(&xmax[b * nao + mu], (unsigned long long)__double_as_longlong(rmax));
  }
}

// ---------------------------------------------------------------------------
// Slicing of X_b (rows mu over k = (P - P0) * nocc + i, stored contiguously by
// the X kernel's blocked layout) into digit planes tiled by 64-wide k steps:
// plane a, block b, step ks holds nao_pad rows of 64 bytes (k = 64 ks .. +63
// in natural order), zero padded; element (a, b, mu, k) sits at
// a plane + ((b nks + k / 64) nao_pad + mu) 64 + k % 64, nks = kbp / 64.  One
// thread per 16 consecutive k; four neighbouring threads fill one 64-byte row.
// ---------------------------------------------------------------------------
template <int S>
__global__ __launch_bounds__(256) void k_slice_x(const double* __restrict__ Xb, int64_t naux,
                                                 int nao, int nocc, int pblk, int nb,
                                                 int nao_pad, int kbp,
                                                 const unsigned long long* __restrict__ xmax,
                                                 int32_t* __restrict__ F,
                                                 int8_t* __restrict__ Xd,
                                                 double* __restrict__ xss) {
  const int nks = kbp >> 6;
  const int64_t total = (int64_t)nb * nks * nao_pad * 4;
  const int64_t plane = (int64_t)nb * nao_pad * kbp;
  const int64_t kfull = (int64_t)pblk * nocc;
  // every thread runs the same number of rounds; with xss given, each wave
  // also sums the squares of its 16 rows x 64 values of X (one aux block, one
  // 64-wide k step: the 64 consecutive idx of a wave) into its own slot
  // xss[idx / 64] (no atomics; total is a multiple of 64)
  for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x; i0 < total;
       i0 += (int64_t)gridDim.x * blockDim.x) {
    const int64_t idx = i0 + threadIdx.x;
    double sq = 0.0;
    if (idx < total) {
    const int part = (int)(idx & 3);
    const int64_t rest = idx >> 2;
    const int mu = (int)(rest % nao_pad);
    const int64_t bks = rest / nao_pad;  // b nks + ks
    const int ks = (int)(bks % nks);
    const int b = (int)(bks / nks);
    const int kc = ks * 4 + part;         // 16-wide k unit within the block
    const int64_t p0 = (int64_t)b * pblk;
    const int64_t p1 = p0 + pblk < naux ? p0 + pblk : naux;
    const int kb = (int)((p1 - p0) * nocc);
    int e = 0;
    if (mu < nao) e = exp_of_max(abs_max_bits_to_double(xmax[(int64_t)b * nao + mu]));
    if (kc == 0) F[(int64_t)b * nao_pad + mu] = e;
    const double* src = Xb + ((int64_t)b * nao + (mu < nao ? mu : 0)) * kfull + kc * 16;
    const bool full = mu < nao && kc * 16 + 16 <= kb;
    // values past the block's k range (and rows past nao) are 0: zero digits
    double v[16];
    if (full) {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const double2 p = *reinterpret_cast<const double2*>(src + 2 * j);
        v[2 * j] = p.x;
        v[2 * j + 1] = p.y;
      }
    } else {
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int k = kc * 16 + j;
        v[j] = (mu < nao && k < kb) ? src[j] : 0.0;
      }
    }
    uint2 r0[S], r1[S];
    digit_rows8<S>(v, e, r0);
    digit_rows8<S>(v + 8, e, r1);
    int8_t* dst = Xd + (bks * nao_pad + mu) * 64 + part * 16;
#pragma unroll
    for (int a = 0; a < S; ++a)
      *reinterpret_cast<uint4*>(dst + (int64_t)a * plane) = make_uint4(r0[a].x, r0[a].y, r1[a].x, r1[a].y);
    if (xss) {
#pragma unroll
      for (int j = 0; j < 16; ++j) sq = fma(v[j], v[j], sq);
    }
    }
    if (xss) {
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) sq += __shfl_xor(sq, off);
      const int64_t w0 = i0 + (threadIdx.x & ~63);
      if ((threadIdx.x & 63) == 0 && w0 < total) xss[w0 >> 6] = sq;
    }
  }
}

__device__ __forceinline__ void lower_tile(int idx, int& t1, int& t2) {
  int r = (int)((sqrtf(8.0f * (float)idx + 1.0f) - 1.0f) * 0.5f);
  while ((r + 1) * (r + 2) / 2 <= idx) ++r;
  while (r * (r + 1) / 2 > idx) --r;
  t1 = r;
  t2 = idx - r * (r + 1) / 2;
}

// ---------------------------------------------------------------------------
// K partials: Kp[grp][mu][nu] = sum over blocks b of group grp (ascending) of
// recombine(S_g of X_b X_b^T), on lower 64x64 tiles; 8 waves x (32 x 16).
// Per 64-wide k step the two row panels (S planes x 64 rows x 64 B each, the
// rows of tile row t1 and of tile column t2) are copied straight from the
// tiled digit planes into one of two LDS stages (buffer loads to LDS, 1 KB =
// 16 rows per wave instruction), while the MFMAs run on the other stage; one
// barrier per step.
// ---------------------------------------------------------------------------
template <int S, bool DBG, int E>
__global__ __launch_bounds__(512) void k_k_int8(const int8_t* __restrict__ Xd,
                                                const int32_t* __restrict__ F, int nb, int nao,
                                                int nao_pad, int kbp, int groups,
                                                double* __restrict__ Kp,
                                                int32_t* __restrict__ dbg) {
  constexpr int ROW = 64;             // 64 B rows, 16-byte units swizzled (swz)
  constexpr int NCP = 2 * S * 4;      // 1 KB copies per step (2 panels x S planes x 4)
  constexpr int CPW = NCP / 8;        // per wave: S, the same for every wave
  static_assert(NCP % 8 == 0, "every wave issues the same number of copies");
  // stages as separate arrays (the compiler can tell the stage being copied
  // into from the one being read); rows [panel][a][64].  Two stages of 16 S KB:
  // two workgroups per CU up to s = 5.
  __shared__ __attribute__((aligned(16))) int8_t L0[2 * S * 64][ROW];
  __shared__ __attribute__((aligned(16))) int8_t L1[2 * S * 64][ROW];
  static_assert(sizeof(L0) + sizeof(L1) <= kLdsLimit, "K stages exceed LDS");
  // group-major logical order, dealt to the XCDs in consecutive ranges: the
  // tiles of one group (which stream the same X_b panels) share an L2
  const int64_t ntile = gridDim.x;
  const int64_t lid = xcd_order(blockIdx.x + (int64_t)blockIdx.y * ntile, ntile * gridDim.y);
  const int grp = (int)(lid / ntile);
  int t1, t2;
  lower_tile((int)(lid - grp * ntile), t1, t2);
  const int b_lo = (int)((int64_t)grp * nb / groups);
  const int b_hi = (int)((int64_t)(grp + 1) * nb / groups);
  const int t = threadIdx.x, w = t >> 6, l = t & 63, q = l >> 4, r16 = l & 15;
  const int wr = (w >> 2) * 32, wc = (w & 3) * 16;
  const int64_t plane = (int64_t)nb * nao_pad * kbp, bstride = (int64_t)nao_pad * kbp;
  const int nks = kbp >> 6;
  // copy j of this wave: panel, plane a, 16-row quarter; lane l lands at byte
  // 16 l of the block (row quarter*16 + l/4, unit l%4), so it fetches the
  // 16-byte unit that the row swizzle puts there
  int cpa[CPW], voff[CPW], crow[CPW];
  const int wu = __builtin_amdgcn_readfirstlane(w);  // wave-uniform copy of w
#pragma unroll
  for (int j = 0; j < CPW; ++j) {
    const int c = wu + 8 * j;  // < NCP
    const int panel = c / (4 * S), a = (c / 4) % S, quarter = c % 4;
    const int row = quarter * 16 + (l >> 2), part = (l & 3) ^ ((row >> 1) & 3);
    cpa[j] = a;
    voff[j] = ((panel ? t2 : t1) * 64 + row) * 64 + part * 16;
    crow[j] = (panel * S + a) * 64 + quarter * 16;
  }
  auto copy_step = [&](auto& L, int b, int ks) {
#pragma unroll
    for (int j = 0; j < CPW; ++j) {
      const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
          const_cast<int8_t*>(Xd + cpa[j] * plane + b * bstride), (short)0, (int)bstride,
          0x00020000);
      copy16_to_lds(r, &L[crow[j]][0], voff[j], ks * nao_pad * 64);
    }
  };

  double kacc[2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) kacc[i][r] = 0.0;
  constexpr int G = S + E;  // anti-diagonals kept (E extra ones)
  i32x4 acc[G][2];
#pragma unroll
  for (int g = 0; g < G; ++g)
#pragma unroll
    for (int i = 0; i < 2; ++i) acc[g][i] = i32x4{0, 0, 0, 0};

  // MFMAs of one step on stage L
  auto mma_step = [&](auto& L) {
    i32x4 bf[S];
#pragma unroll
    for (int bb = 0; bb < S; ++bb)
      bf[bb] = *reinterpret_cast<const i32x4*>(&L[(S + bb) * 64 + wc + r16][swz(wc + r16, q)]);
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      i32x4 af[S];
      const int row = wr + i * 16 + r16;
#pragma unroll
      for (int a = 0; a < S; ++a)
        af[a] = *reinterpret_cast<const i32x4*>(&L[a * 64 + row][swz(row, q)]);
#pragma unroll
      for (int a = 0; a < S; ++a)
#pragma unroll
        for (int bb = 0; bb < (S - a + E < S ? S - a + E : S); ++bb)
          acc[a + bb][i] = __builtin_amdgcn_mfma_i32_16x16x64_i8(af[a], bf[bb], acc[a + bb][i], 0, 0, 0);
    }
  };
  // end of aux block b: recombine into the FP64 partial sum
  auto close_block = [&](int b) {
    const int32_t* Fb = F + (int64_t)b * nao_pad;
    const int fn = Fb[t2 * 64 + wc + r16];
    if constexpr (DBG) {  // test export: the int32 anti-diagonal sums of block b on this tile
      const int nu = t2 * 64 + wc + r16;
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int mu = t1 * 64 + wr + i * 16 + q * 4 + r;
          if (mu < nao && nu < nao) {
#pragma unroll
            for (int g = 0; g < G; ++g)
              dbg[(((int64_t)g * nb + b) * nao + mu) * nao + nu] = acc[g][i][r];
          }
        }
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int base = Fb[t1 * 64 + wr + i * 16 + q * 4 + r] + fn + 4;
        double z = 0.0;
#pragma unroll
        for (int g = G + 1; g >= 2; --g) z += ldexp((double)acc[g - 2][i][r], base - 8 * g);
        kacc[i][r] += z;
      }
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
      for (int i = 0; i < 2; ++i) acc[g][i] = i32x4{0, 0, 0, 0};
  };

  // steps (b, ks) in order; step n uses stage n % 2
  int b = b_lo, ks = 0;
  if (b < b_hi) copy_step(L0, b, 0);
  __syncthreads();
  while (b < b_hi) {
    // even step on L0, the next one copied into L1
    {
      const int nb_ = ks + 1 == nks ? b + 1 : b, nk_ = ks + 1 == nks ? 0 : ks + 1;
      if (nb_ < b_hi) copy_step(L1, nb_, nk_);
      mma_step(L0);
      if (ks + 1 == nks) close_block(b);
      __syncthreads();  // L0 may be overwritten; this wave's copies into L1 have landed
      b = nb_;
      ks = nk_;
    }
    if (b >= b_hi) break;
    // odd step on L1, the next one copied into L0
    {
      const int nb_ = ks + 1 == nks ? b + 1 : b, nk_ = ks + 1 == nks ? 0 : ks + 1;
      if (nb_ < b_hi) copy_step(L0, nb_, nk_);
      mma_step(L1);
      if (ks + 1 == nks) close_block(b);
      __syncthreads();
      b = nb_;
      ks = nk_;
    }
  }

  double* out = Kp + (int64_t)grp * nao * nao;
  const int nu = t2 * 64 + wc + r16;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int mu = t1 * 64 + wr + i * 16 + q * 4 + r;
      if (mu < nao && nu < nao) out[(int64_t)mu * nao + nu] = kacc[i][r];
    }
}

// ---------------------------------------------------------------------------
// Test hook: one kept pair (a, b) per z-slice of the grid, one 16x16 tile per
// wave, operands padded to [s][rows_pad][k_pad] with k in natural order.
// ---------------------------------------------------------------------------
__global__ void k_pad_rows(const int8_t* __restrict__ src, int64_t rows, int64_t k, int s,
                           int64_t rows_pad, int64_t k_pad, int transpose,
                           int8_t* __restrict__ dst) {
  const int64_t n = (int64_t)s * rows_pad * k_pad;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t kk = idx % k_pad;
    const int64_t rest = idx / k_pad;
    const int64_t r = rest % rows_pad;
    const int64_t a = rest / rows_pad;
    int8_t v = 0;
    if (r < rows && kk < k)
      v = transpose ? src[(a * k + kk) * rows + r] : src[(a * rows + r) * k + kk];
    dst[idx] = v;
  }
}

__global__ __launch_bounds__(64) void k_debug_pairs(const int8_t* __restrict__ A,
                                                    const int8_t* __restrict__ Bt, int64_t m,
                                                    int64_t n, int64_t m_pad, int64_t n_pad,
                                                    int64_t k_pad, int s,
                                                    int32_t* __restrict__ partials) {
  const int l = threadIdx.x;
  const int p = blockIdx.z;
  int a = 0, b = 0, cnt = 0;
  for (int aa = 0; aa < s; ++aa)
    for (int bb = 0; bb < s - aa; ++bb) {
      if (cnt == p) { a = aa; b = bb; }
      ++cnt;
    }
  const int64_t r0 = (int64_t)blockIdx.x * 16, c0 = (int64_t)blockIdx.y * 16;
  const int8_t* pa = A + ((int64_t)a * m_pad + r0 + (l & 15)) * k_pad + (l >> 4) * 16;
  const int8_t* pb = Bt + ((int64_t)b * n_pad + c0 + (l & 15)) * k_pad + (l >> 4) * 16;
  i32x4 acc = {0, 0, 0, 0};
  for (int64_t k0 = 0; k0 < k_pad; k0 += 64) {
    const i32x4 fa = *reinterpret_cast<const i32x4*>(pa + k0);
    const i32x4 fb = *reinterpret_cast<const i32x4*>(pb + k0);
    acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(fa, fb, acc, 0, 0, 0);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int64_t row = r0 + (l >> 4) * 4 + r, col = c0 + (l & 15);
    if (row < m && col < n) partials[((int64_t)p * m + row) * n + col] = acc[r];
  }
}

template <int S, bool FULLK, int KSUB, bool PK = false, int E = 0>
hipError_t launch_x_sk(hipStream_t st, const double* B, int64_t M, int nao, const int32_t* b_exp,
                       const int8_t* dC, int ncp, int kp, const int32_t* f_col, int nocc,
                       double* X, int xlayout, unsigned long long* xmax, int pblk, const double* D,
                       double* rowdot, const unsigned long long* cmask, int32_t* dbg) {
  // PK: one tile per (P, 64 rows of B_P); else 64 consecutive rows of the
  // stacked (P, mu) rows
  const unsigned gx = PK ? (unsigned)(M / nao * ((nao + 63) / 64)) : (unsigned)((M + 63) / 64);
#define DFJK_XK(NF_)                                                                             \
  hipLaunchKernelGGL((k_x_int8<S, NF_, FULLK, KSUB, PK, E>), dim3(gx, ncp / (16 * (NF_))),        \
                     dim3(512), 0, st, B, M, nao, b_exp, dC, ncp, kp, f_col, nocc, X, xlayout, xmax, \
                     nao, pblk, D, rowdot, cmask, dbg)
  // one column tile over 128 or 192 columns where the stages fit in LDS (B is
  // then read and sliced once), else tiles of 96, 64 or 32 columns
  if constexpr (S <= 4 && KSUB == 1) {
    if (ncp == 192) {
      DFJK_XK(12);
      return hipGetLastError();
    }
  }
  if constexpr (S + E <= 6 && KSUB == 1) {
    if (ncp == 128) {
      DFJK_XK(8);
      return hipGetLastError();
    }
  }
  if (ncp % 96 == 0) DFJK_XK(6);
  else if (ncp % 64 == 0) DFJK_XK(4);
  else DFJK_XK(2);
#undef DFJK_XK
  return hipGetLastError();
}

// Chunks of 128 k (two MFMA k steps, one LDS stage) only when asked for
// (ksub = 2, an autotuner choice; s <= 5 and nao a multiple of 128); by default
// 64-wide chunks in two LDS stages with direct C copies and buffer loads.
template <int S>
hipError_t launch_x_s(hipStream_t st, const double* B, int64_t M, int nao, const int32_t* b_exp,
                      const int8_t* dC, int ncp, int kp, const int32_t* f_col, int nocc,
                      double* X, int xlayout, unsigned long long* xmax, int pblk, const double* D,
                      double* rowdot, const unsigned long long* cmask, int ksub, int32_t* dbg,
                      int packed, int extra) {
  if (S > 1 && extra) {  // one extra anti-diagonal: 64-wide chunks
    if (packed)
      return launch_x_sk<S, true, 1, true, 1>(st, B, M, nao, b_exp, dC, ncp, kp, f_col, nocc, X,
                                              xlayout, xmax, pblk, D, rowdot, nullptr, dbg);
    if (nao % 64 == 0)
      return launch_x_sk<S, true, 1, false, 1>(st, B, M, nao, b_exp, dC, ncp, kp, f_col, nocc, X,
                                               xlayout, xmax, pblk, D, rowdot, cmask, dbg);
    return launch_x_sk<S, false, 1, false, 1>(st, B, M, nao, b_exp, dC, ncp, kp, f_col, nocc, X,
                                              xlayout, xmax, pblk, D, rowdot, cmask, dbg);
  }
  if (packed)  // 64-wide chunks; no screening masks
    return launch_x_sk<S, true, 1, true>(st, B, M, nao, b_exp, dC, ncp, kp, f_col, nocc, X, xlayout,
                                         xmax, pblk, D, rowdot, nullptr, dbg);
  if (S <= 5 && nao % 128 == 0 && ksub == 2)
    return launch_x_sk<S, true, (S <= 5 ? 2 : 1)>(st, B, M, nao, b_exp, dC, ncp, kp, f_col, nocc, X,
                                                   xlayout, xmax, pblk, D, rowdot, cmask, dbg);
  if (nao % 64 == 0)
    return launch_x_sk<S, true, 1>(st, B, M, nao, b_exp, dC, ncp, kp, f_col, nocc, X, xlayout, xmax,
                                   pblk, D, rowdot, cmask, dbg);
  return launch_x_sk<S, false, 1>(st, B, M, nao, b_exp, dC, ncp, kp, f_col, nocc, X, xlayout, xmax,
                                  pblk, D, rowdot, cmask, dbg);
}

}  // namespace

hipError_t launch_x_int8(hipStream_t st, int s, const double* B, int64_t naux, int nao,
                         const int32_t* b_exp, const int8_t* dC, int ncp, int kp,
                         const int32_t* f_col, int nocc, double* X, int xlayout,
                         unsigned long long* xmax, int pblk, const double* D, double* rowdot,
                         const unsigned long long* cmask, int ksub, int32_t* dbg, int packed,
                         int extra) {
  const int64_t M = naux * nao;
  if (M <= 0 || nocc <= 0) return hipSuccess;
  switch (s) {
    case 1: return launch_x_s<1>(st, B, M, nao, b_exp, dC, ncp, kp, f_col, nocc, X, xlayout, xmax, pblk, D, rowdot, cmask, ksub, dbg, packed, extra);
    case 2: return launch_x_s<2>(st, B, M, nao, b_exp, dC, ncp, kp, f_col, nocc, X, xlayout, xmax, pblk, D, rowdot, cmask, ksub, dbg, packed, extra);
    case 3: return launch_x_s<3>(st, B, M, nao, b_exp, dC, ncp, kp, f_col, nocc, X, xlayout, xmax, pblk, D, rowdot, cmask, ksub, dbg, packed, extra);
    case 4: return launch_x_s<4>(st, B, M, nao, b_exp, dC, ncp, kp, f_col, nocc, X, xlayout, xmax, pblk, D, rowdot, cmask, ksub, dbg, packed, extra);
    case 5: return launch_x_s<5>(st, B, M, nao, b_exp, dC, ncp, kp, f_col, nocc, X, xlayout, xmax, pblk, D, rowdot, cmask, ksub, dbg, packed, extra);
    case 6: return launch_x_s<6>(st, B, M, nao, b_exp, dC, ncp, kp, f_col, nocc, X, xlayout, xmax, pblk, D, rowdot, cmask, ksub, dbg, packed, extra);
    case 7: return launch_x_s<7>(st, B, M, nao, b_exp, dC, ncp, kp, f_col, nocc, X, xlayout, xmax, pblk, D, rowdot, cmask, ksub, dbg, packed, extra);
    case 8: return launch_x_s<8>(st, B, M, nao, b_exp, dC, ncp, kp, f_col, nocc, X, xlayout, xmax, pblk, D, rowdot, cmask, ksub, dbg, packed, extra);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_slice_x(hipStream_t st, int s, const double* X, int64_t naux, int nao,
                          int nocc, int pblk, int nao_pad, int kbp,
                          const unsigned long long* xmax, int32_t* F, int8_t* Xd, double* xss) {
  const int nb = (int)((naux + pblk - 1) / pblk);
  const int64_t total = (int64_t)nb * nao_pad * (kbp / 16);  // threads (16 k each)
  if (total <= 0) return hipSuccess;
  int64_t g = (total + 255) / 256;
  if (g > 65536) g = 65536;
#define DFJK_SLICE_X(SS)                                                                      \
  hipLaunchKernelGGL((k_slice_x<SS>), dim3((unsigned)g), dim3(256), 0, st, X, naux, nao, nocc, \
                     pblk, nb, nao_pad, kbp, xmax, F, Xd, xss)
  switch (s) {
    case 1: DFJK_SLICE_X(1); break;
    case 2: DFJK_SLICE_X(2); break;
    case 3: DFJK_SLICE_X(3); break;
    case 4: DFJK_SLICE_X(4); break;
    case 5: DFJK_SLICE_X(5); break;
    case 6: DFJK_SLICE_X(6); break;
    case 7: DFJK_SLICE_X(7); break;
    case 8: DFJK_SLICE_X(8); break;
    default: return hipErrorInvalidValue;
  }
#undef DFJK_SLICE_X
  return hipGetLastError();
}

int k_int8_resident(int s) {
  static int cached[9] = {0};  // per slice count (the same on every MI355X)
  if (s < 1 || s > 8) return 1;
  if (cached[s] > 0) return cached[s];
  int n = 0;
  hipError_t e = hipErrorInvalidValue;
#define DFJK_KOCC(SS) \
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void*>(&k_k_int8<SS, false, 0>), 512, 0)
  switch (s) {
    case 1: DFJK_KOCC(1); break;
    case 2: DFJK_KOCC(2); break;
    case 3: DFJK_KOCC(3); break;
    case 4: DFJK_KOCC(4); break;
    case 5: DFJK_KOCC(5); break;
    case 6: DFJK_KOCC(6); break;
    case 7: DFJK_KOCC(7); break;
    case 8: DFJK_KOCC(8); break;
    default: break;
  }
#undef DFJK_KOCC
  if (e != hipSuccess) (void)hipGetLastError();  // leave no error for the next launch check
  cached[s] = e == hipSuccess && n > 0 ? n : 1;
  return cached[s];
}

hipError_t launch_k_int8(hipStream_t st, int s, const int8_t* Xd, const int32_t* F, int nb,
                         int nao, int nao_pad, int kbp, int groups, double* Kp, int32_t* dbg,
                         int extra) {
  const int nt = nao_pad / 64;
  const dim3 grid((unsigned)(nt * (nt + 1) / 2), (unsigned)groups);
#define DFJK_K(SS)                                                                            \
  if (SS > 1 && extra && dbg)                                                                 \
    hipLaunchKernelGGL((k_k_int8<SS, true, (SS > 1 ? 1 : 0)>), grid, dim3(512), 0, st, Xd, F, nb, \
                       nao, nao_pad, kbp, groups, Kp, dbg);                                   \
  else if (SS > 1 && extra)                                                                   \
    hipLaunchKernelGGL((k_k_int8<SS, false, (SS > 1 ? 1 : 0)>), grid, dim3(512), 0, st, Xd, F, nb, \
                       nao, nao_pad, kbp, groups, Kp, nullptr);                               \
  else if (dbg)                                                                               \
    hipLaunchKernelGGL((k_k_int8<SS, true, 0>), grid, dim3(512), 0, st, Xd, F, nb, nao, nao_pad, \
                       kbp, groups, Kp, dbg);                                                 \
  else                                                                                        \
    hipLaunchKernelGGL((k_k_int8<SS, false, 0>), grid, dim3(512), 0, st, Xd, F, nb, nao, nao_pad, \
                       kbp, groups, Kp, nullptr)
  switch (s) {
    case 1: DFJK_K(1); break;
    case 2: DFJK_K(2); break;
    case 3: DFJK_K(3); break;
    case 4: DFJK_K(4); break;
    case 5: DFJK_K(5); break;
    case 6: DFJK_K(6); break;
    case 7: DFJK_K(7); break;
    case 8: DFJK_K(8); break;
    default: return hipErrorInvalidValue;
  }
#undef DFJK_K
  return hipGetLastError();
}

hipError_t launch_debug_pairs(hipStream_t st, int s, const int8_t* a_dig, const int8_t* b_dig,
                              int64_t m, int64_t n, int64_t k, int8_t* ws_a, int8_t* ws_b,
                              int32_t* partials) {
  const int64_t m_pad = (m + 63) / 64 * 64, n_pad = (n + 63) / 64 * 64;
  const int64_t k_pad = (k + 63) / 64 * 64;
  const int64_t na = (int64_t)s * m_pad * k_pad, nbb = (int64_t)s * n_pad * k_pad;
  hipLaunchKernelGGL(k_pad_rows, dim3((unsigned)((na + 255) / 256 > 65536 ? 65536 : (na + 255) / 256)),
                     dim3(256), 0, st, a_dig, m, k, s, m_pad, k_pad, 0, ws_a);
  hipLaunchKernelGGL(k_pad_rows, dim3((unsigned)((nbb + 255) / 256 > 65536 ? 65536 : (nbb + 255) / 256)),
                     dim3(256), 0, st, b_dig, n, k, s, n_pad, k_pad, 1, ws_b);
  const int npairs = s * (s + 1) / 2;
  hipLaunchKernelGGL(k_debug_pairs, dim3((unsigned)(m_pad / 16), (unsigned)(n_pad / 16), npairs),
                     dim3(64), 0, st, ws_a, ws_b, m, n, m_pad, n_pad, k_pad, s, partials);
  return hipGetLastError();
}

}  // namespace dfjk
