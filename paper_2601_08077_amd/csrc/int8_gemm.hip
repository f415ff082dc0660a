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

__device__ __forceinline__ uint32_t pack4(uint64_t w0, uint64_t w1, uint64_t w2, uint64_t w3,
                                          int k) {
  return digit_byte(w0, k) | (digit_byte(w1, k) << 8) | (digit_byte(w2, k) << 16) |
         (digit_byte(w3, k) << 24);
}

// ---------------------------------------------------------------------------
// X = B C.  Tile: 64 rows of (P, mu) x 16*NF columns i; 4 waves x 16 rows.
// Loader: thread t owns row t/4 and lane-group q = t%4 of each 64-wide k chunk;
// it reads 8 double pairs at k = 8 j + 2 q + {0, 1}, so each row segment of
// 64 B is read by 4 consecutive threads.  Slot 2 j + h of group q holds
// k = 8 j + 2 q + h; the C digit planes are stored in the same slot order.
// ---------------------------------------------------------------------------
template <int S, int NF>
__global__ __launch_bounds__(256) void k_x_int8(
    const double* __restrict__ B, int64_t M, int K, const int32_t* __restrict__ b_exp,
    const int8_t* __restrict__ dC, int ncp, int kp, const int32_t* __restrict__ f_col, int nocc,
    double* __restrict__ X, unsigned long long* __restrict__ xmax, int nao, int pblk) {
  constexpr int ROWS = 64, KC = 64, LDS_ROW = 80;  // 16 B pad: conflict-free b128 reads
  __shared__ __attribute__((aligned(16))) int8_t As[S][ROWS][LDS_ROW];

  const int t = threadIdx.x, w = t >> 6, l = t & 63;
  const int64_t m0 = (int64_t)blockIdx.x * ROWS;
  const int n0 = blockIdx.y * 16 * NF;

  const int lr = t >> 2, lq = t & 3;
  const int64_t grow = m0 + lr;
  const bool row_ok = grow < M;
  const double* brow = B + (row_ok ? grow : 0) * (int64_t)K;
  const int e_ld = row_ok ? b_exp[grow] : 0;
  const bool even_k = (K & 1) == 0;

  i32x4 acc[S][NF];
#pragma unroll
  for (int g = 0; g < S; ++g)
#pragma unroll
    for (int f = 0; f < NF; ++f) acc[g][f] = i32x4{0, 0, 0, 0};

  const int nchunks = (K + KC - 1) / KC;
  for (int c = 0; c < nchunks; ++c) {
    const int k0 = c * KC;
    uint64_t wd[16];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int kk = k0 + 8 * j + 2 * lq;
      double v0 = 0.0, v1 = 0.0;
      if (row_ok) {
        if (even_k && kk + 1 < K) {
          const double2 p = *reinterpret_cast<const double2*>(brow + kk);
          v0 = p.x;
          v1 = p.y;
        } else {
          if (kk < K) v0 = brow[kk];
          if (kk + 1 < K) v1 = brow[kk + 1];
        }
      }
      wd[2 * j] = digit_word(v0, e_ld);
      wd[2 * j + 1] = digit_word(v1, e_ld);
    }
    __syncthreads();
#pragma unroll
    for (int a = 0; a < S; ++a) {
      uint4 pk;
      pk.x = pack4(wd[0], wd[1], wd[2], wd[3], a + 1);
      pk.y = pack4(wd[4], wd[5], wd[6], wd[7], a + 1);
      pk.z = pack4(wd[8], wd[9], wd[10], wd[11], a + 1);
      pk.w = pack4(wd[12], wd[13], wd[14], wd[15], a + 1);
      *reinterpret_cast<uint4*>(&As[a][lr][lq * 16]) = pk;
    }
    __syncthreads();

    i32x4 af[S];
#pragma unroll
    for (int a = 0; a < S; ++a)
      af[a] = *reinterpret_cast<const i32x4*>(&As[a][w * 16 + (l & 15)][(l >> 4) * 16]);
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      const int8_t* cb = dC + (int64_t)(n0 + f * 16 + (l & 15)) * kp + k0 + (l >> 4) * 16;
      i32x4 bf[S];
#pragma unroll
      for (int b = 0; b < S; ++b)
        bf[b] = *reinterpret_cast<const i32x4*>(cb + (int64_t)b * ncp * kp);
#pragma unroll
      for (int a = 0; a < S; ++a)
#pragma unroll
        for (int b = 0; b < S - a; ++b)
          acc[a + b][f] = __builtin_amdgcn_mfma_i32_16x16x64_i8(af[a], bf[b], acc[a + b][f], 0, 0, 0);
    }
  }

  // Recombination, X store, and the per-(block, mu) running max of |X|.
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int64_t row = m0 + w * 16 + (l >> 4) * 4 + r;
    const bool vr = row < M;
    const int er = vr ? b_exp[row] : 0;
    double rmax = 0.0;
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      const int col = n0 + f * 16 + (l & 15);
      if (vr && col < nocc) {
        const int base = er + f_col[col] + 4;
        double z = 0.0;
#pragma unroll
        for (int g = S + 1; g >= 2; --g) z += ldexp((double)acc[g - 2][f][r], base - 8 * g);
        X[row * nocc + col] = z;
        rmax = fmax(rmax, fabs(z));
      }
    }
#pragma unroll
    for (int off = 1; off < 16; off <<= 1) rmax = fmax(rmax, __shfl_xor(rmax, off));
    if ((l & 15) == 0 && vr) {
      const int64_t P = row / nao;
      const int mu = (int)(row - P * nao);
      const int64_t b = P / pblk;
      atomicMax(&xmax[b * nao + mu], (unsigned long long)__double_as_longlong(rmax));
    }
  }
}

// ---------------------------------------------------------------------------
// Slicing of X_b (rows mu over k = (P - P0) * nocc + i) into Xd[a][b][mu][k],
// natural k order, zero padded to nao_pad rows and kbp columns.  One thread
// per 16 consecutive k of one (b, mu).
// ---------------------------------------------------------------------------
template <int S>
__global__ __launch_bounds__(256) void k_slice_x(const double* __restrict__ X, int64_t naux,
                                                 int nao, int nocc, int pblk, int nb,
                                                 int nao_pad, int kbp,
                                                 const unsigned long long* __restrict__ xmax,
                                                 int32_t* __restrict__ F,
                                                 int8_t* __restrict__ Xd) {
  const int nkc = kbp >> 4;
  const int64_t total = (int64_t)nb * nao_pad * nkc;
  const int64_t plane = (int64_t)nb * nao_pad * kbp;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int kc = (int)(idx % nkc);
    const int64_t rest = idx / nkc;
    const int mu = (int)(rest % nao_pad);
    const int b = (int)(rest / nao_pad);
    const int64_t p0 = (int64_t)b * pblk;
    const int64_t p1 = p0 + pblk < naux ? p0 + pblk : naux;
    const int kb = (int)(p1 - p0) * nocc;
    int e = 0;
    if (mu < nao) e = exp_of_max(abs_max_bits_to_double(xmax[(int64_t)b * nao + mu]));
    if (kc == 0) F[(int64_t)b * nao_pad + mu] = e;
    uint64_t wd[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int k = kc * 16 + j;
      double v = 0.0;
      if (mu < nao && k < kb) {
        const int pp = k / nocc, i = k - pp * nocc;
        v = X[((p0 + pp) * nao + mu) * (int64_t)nocc + i];
      }
      wd[j] = digit_word(v, e);
    }
    int8_t* dst = Xd + ((int64_t)b * nao_pad + mu) * kbp + kc * 16;
#pragma unroll
    for (int a = 0; a < S; ++a) {
      uint4 pk;
      pk.x = pack4(wd[0], wd[1], wd[2], wd[3], a + 1);
      pk.y = pack4(wd[4], wd[5], wd[6], wd[7], a + 1);
      pk.z = pack4(wd[8], wd[9], wd[10], wd[11], a + 1);
      pk.w = pack4(wd[12], wd[13], wd[14], wd[15], a + 1);
      *reinterpret_cast<uint4*>(dst + (int64_t)a * plane) = pk;
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
// recombine(S_g of X_b X_b^T), on lower 64x64 tiles; 4 waves x (32 x 32).
// ---------------------------------------------------------------------------
template <int S>
__global__ __launch_bounds__(256) void k_k_int8(const int8_t* __restrict__ Xd,
                                                const int32_t* __restrict__ F, int nb, int nao,
                                                int nao_pad, int kbp, int groups,
                                                double* __restrict__ Kp) {
  int t1, t2;
  lower_tile(blockIdx.x, t1, t2);
  const int grp = blockIdx.y;
  const int b_lo = (int)((int64_t)grp * nb / groups);
  const int b_hi = (int)((int64_t)(grp + 1) * nb / groups);
  const int t = threadIdx.x, w = t >> 6, l = t & 63;
  const int rbase = t1 * 64 + (w >> 1) * 32;
  const int cbase = t2 * 64 + (w & 1) * 32;
  const int64_t plane = (int64_t)nb * nao_pad * kbp;

  double kacc[2][2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) kacc[i][j][r] = 0.0;

  for (int b = b_lo; b < b_hi; ++b) {
    i32x4 acc[S][2][2];
#pragma unroll
    for (int g = 0; g < S; ++g)
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[g][i][j] = i32x4{0, 0, 0, 0};

    const int8_t* xb = Xd + (int64_t)b * nao_pad * kbp;
    const int8_t* ra0 = xb + (int64_t)(rbase + (l & 15)) * kbp + (l >> 4) * 16;
    const int8_t* ra1 = ra0 + 16 * (int64_t)kbp;
    const int8_t* ca0 = xb + (int64_t)(cbase + (l & 15)) * kbp + (l >> 4) * 16;
    const int8_t* ca1 = ca0 + 16 * (int64_t)kbp;
    for (int k0 = 0; k0 < kbp; k0 += 64) {
      i32x4 af[S][2], bf[S][2];
#pragma unroll
      for (int a = 0; a < S; ++a) {
        af[a][0] = *reinterpret_cast<const i32x4*>(ra0 + a * plane + k0);
        af[a][1] = *reinterpret_cast<const i32x4*>(ra1 + a * plane + k0);
        bf[a][0] = *reinterpret_cast<const i32x4*>(ca0 + a * plane + k0);
        bf[a][1] = *reinterpret_cast<const i32x4*>(ca1 + a * plane + k0);
      }
#pragma unroll
      for (int a = 0; a < S; ++a)
#pragma unroll
        for (int bb = 0; bb < S - a; ++bb)
#pragma unroll
          for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
              acc[a + bb][i][j] =
                  __builtin_amdgcn_mfma_i32_16x16x64_i8(af[a][i], bf[bb][j], acc[a + bb][i][j], 0, 0, 0);
    }
    const int32_t* Fb = F + (int64_t)b * nao_pad;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int nu = cbase + j * 16 + (l & 15);
        const int fn = Fb[nu];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int mu = rbase + i * 16 + (l >> 4) * 4 + r;
          const int base = Fb[mu] + fn + 4;
          double z = 0.0;
#pragma unroll
          for (int g = S + 1; g >= 2; --g) z += ldexp((double)acc[g - 2][i][j][r], base - 8 * g);
          kacc[i][j][r] += z;
        }
      }
  }

  double* out = Kp + (int64_t)grp * nao * nao;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int nu = cbase + j * 16 + (l & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int mu = rbase + i * 16 + (l >> 4) * 4 + r;
        if (mu < nao && nu < nao) out[(int64_t)mu * nao + nu] = kacc[i][j][r];
      }
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

template <int S>
hipError_t launch_x_s(hipStream_t st, const double* B, int64_t M, int nao, const int32_t* b_exp,
                      const int8_t* dC, int ncp, int kp, const int32_t* f_col, int nocc,
                      double* X, unsigned long long* xmax, int pblk) {
  const unsigned gx = (unsigned)((M + 63) / 64);
  if (ncp % 96 == 0) {
    hipLaunchKernelGGL((k_x_int8<S, 6>), dim3(gx, ncp / 96), dim3(256), 0, st, B, M, nao, b_exp,
                       dC, ncp, kp, f_col, nocc, X, xmax, nao, pblk);
  } else if (ncp % 64 == 0) {
    hipLaunchKernelGGL((k_x_int8<S, 4>), dim3(gx, ncp / 64), dim3(256), 0, st, B, M, nao, b_exp,
                       dC, ncp, kp, f_col, nocc, X, xmax, nao, pblk);
  } else {
    hipLaunchKernelGGL((k_x_int8<S, 2>), dim3(gx, ncp / 32), dim3(256), 0, st, B, M, nao, b_exp,
                       dC, ncp, kp, f_col, nocc, X, xmax, nao, pblk);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_x_int8(hipStream_t st, int s, const double* B, int64_t naux, int nao,
                         const int32_t* b_exp, const int8_t* dC, int ncp, int kp,
                         const int32_t* f_col, int nocc, double* X, unsigned long long* xmax,
                         int pblk) {
  const int64_t M = naux * nao;
  if (M <= 0 || nocc <= 0) return hipSuccess;
  switch (s) {
    case 1: return launch_x_s<1>(st, B, M, nao, b_exp, dC, ncp, kp, f_col, nocc, X, xmax, pblk);
    case 2: return launch_x_s<2>(st, B, M, nao, b_exp, dC, ncp, kp, f_col, nocc, X, xmax, pblk);
    case 3: return launch_x_s<3>(st, B, M, nao, b_exp, dC, ncp, kp, f_col, nocc, X, xmax, pblk);
    case 4: return launch_x_s<4>(st, B, M, nao, b_exp, dC, ncp, kp, f_col, nocc, X, xmax, pblk);
    case 5: return launch_x_s<5>(st, B, M, nao, b_exp, dC, ncp, kp, f_col, nocc, X, xmax, pblk);
    case 6: return launch_x_s<6>(st, B, M, nao, b_exp, dC, ncp, kp, f_col, nocc, X, xmax, pblk);
    case 7: return launch_x_s<7>(st, B, M, nao, b_exp, dC, ncp, kp, f_col, nocc, X, xmax, pblk);
    case 8: return launch_x_s<8>(st, B, M, nao, b_exp, dC, ncp, kp, f_col, nocc, X, xmax, pblk);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_slice_x(hipStream_t st, int s, const double* X, int64_t naux, int nao,
                          int nocc, int pblk, int nao_pad, int kbp,
                          const unsigned long long* xmax, int32_t* F, int8_t* Xd) {
  const int nb = (int)((naux + pblk - 1) / pblk);
  const int64_t total = (int64_t)nb * nao_pad * (kbp / 16);
  if (total <= 0) return hipSuccess;
  int64_t g = (total + 255) / 256;
  if (g > 65536) g = 65536;
#define DFJK_SLICE_X(SS)                                                                      \
  hipLaunchKernelGGL((k_slice_x<SS>), dim3((unsigned)g), dim3(256), 0, st, X, naux, nao, nocc, \
                     pblk, nb, nao_pad, kbp, xmax, F, Xd)
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

hipError_t launch_k_int8(hipStream_t st, int s, const int8_t* Xd, const int32_t* F, int nb,
                         int nao, int nao_pad, int kbp, int groups, double* Kp) {
  const int nt = nao_pad / 64;
  const dim3 grid((unsigned)(nt * (nt + 1) / 2), (unsigned)groups);
#define DFJK_K(SS) \
  hipLaunchKernelGGL((k_k_int8<SS>), grid, dim3(256), 0, st, Xd, F, nb, nao, nao_pad, kbp, groups, Kp)
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
