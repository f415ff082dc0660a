// Native FP64 path of the exchange build (the paper's level 0 / standard FP64,
// Table 1 and Sec. 3.2) on gfx950 v_mfma_f64_16x16x4_f64.
//
// MFMA operand layout (checked on gfx950): lane l holds A[l & 15][l >> 4] and
// B[l >> 4][l & 15]; result register r of lane l is row 4 r + (l >> 4),
// column (l & 15).
#include "dfjk_internal.h"

namespace dfjk {
namespace {

__device__ __forceinline__ f64x4 mfma_f64(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// X = B C (Eq. 5): 64 rows (P, mu) x 16*NF columns per workgroup, k chunks of
// 16 staged through LDS; 4 waves x 16 rows.  Also the per-(block, mu) max |X|
// and, when D is given, the row dots sum_nu B[P][mu][nu] D[mu][nu] (Eq. 3).
// X layout 0: X[row][i]; 1: blocked (X_b rows mu over (P - P0, i)).
//
// Dense B: thread t loads 4 consecutive k of tile row t / 4 (two 16-byte loads
// on the full path, nao a multiple of 16 and no screening).  Packed B (PK;
// B_P stored as its lower triangle by rows): one tile per (P, 64 rows of
// B_P), and each 16-wide k step of the tile is one of three kinds: entirely
// below its rows (the rows of the triangle, read like dense rows), entirely
// above them (the mirrored block: stored rows nu over the tile's mu, so thread
// t loads column group t / 64 of tile row t % 64 and every load instruction
// reads 64 consecutive mu of one stored row), or across the diagonal (element
// by element).  The values reaching the MFMAs are the same in every case.
// With PK the row dots cover the steps up to the diagonal only (B_P and D are
// symmetric: below counted twice, across the diagonal by element with weights
// 2 / 1 / 0): the same sum in another rounding order.
template <int NF, bool PK, bool VEC>
__global__ __launch_bounds__(256) void k_x_fp64(const double* __restrict__ B, int64_t M, int K,
                                                const double* __restrict__ C, int nocc,
                                                double* __restrict__ X, int xlayout,
                                                unsigned long long* __restrict__ xmax, int nao,
                                                int pblk, const double* __restrict__ D,
                                                double* __restrict__ rowdot,
                                                const unsigned long long* __restrict__ cmask) {
  constexpr int NT = 16 * NF;
  __shared__ double As[2][64][17];
  __shared__ double Cs[2][16][NT + 1];
  const int t = threadIdx.x, w = t >> 6, l = t & 63;
  int64_t m0 = (int64_t)blockIdx.x * 64;
  int64_t ptile = 0;
  int mu0 = 0;
  if constexpr (PK) {
    // the tiles of one P are consecutive and go to one XCD (their mirrored
    // reads of one stored block meet in L2)
    const int nmt = (nao + 63) >> 6;
    const int64_t lid = xcd_order(blockIdx.x, gridDim.x);
    ptile = lid / nmt;
    mu0 = (int)(lid - ptile * nmt) * 64;
    m0 = ptile * nao + mu0;
  } else if (nao % 64 == 0) {
    // workgroups that run together share the basis-row tile (and the rows of
    // D) and differ in the aux index P
    const int64_t naux = M / nao;
    const int64_t mt = blockIdx.x / naux, P = blockIdx.x - mt * naux;
    m0 = P * nao + mt * 64;
  }
  const int n0 = blockIdx.y * NT;

  const int lr = t >> 2, lk = (t & 3) * 4;      // row-wise loader: tile row, k offset
  const int lrT = t & 63, lkT = (t >> 6) * 4;   // mirrored loader (PK)
  const int64_t grow = m0 + lr;
  const bool row_ok = PK ? mu0 + lr < nao : grow < M;
  const int mu = PK ? min(mu0 + lr, nao - 1) : 0;  // padding rows read row nao - 1
  const int muT = PK ? min(mu0 + lrT, nao - 1) : 0;
  const double* bpk = B + (PK ? ptile * ((int64_t)nao * (nao + 1) / 2) : 0);
  const int64_t tri_mu = (int64_t)mu * (mu + 1) / 2;
  const double* brow = PK ? bpk + tri_mu : B + (row_ok ? grow : 0) * (int64_t)K;
  const double* drow =
      D ? D + (row_ok ? (PK ? (int64_t)(mu0 + lr) : grow % nao) : 0) * (int64_t)K : nullptr;
  double rd = 0.0;

  f64x4 acc[NF];
#pragma unroll
  for (int f = 0; f < NF; ++f) acc[f] = f64x4{0.0, 0.0, 0.0, 0.0};

  // Register sets of one 16-k chunk: B values, C values, D values of the row
  // dots, and (PK) the chunk's kind.  Two sets: the loads of chunk c + 2 are
  // issued while chunk c is multiplied, so every load has two chunks of
  // MFMAs to land (the D values travel with the chunk, so that no later load
  // is waited on before them).
  struct Regs {
    double va[4], vc[NF], vd[4];
    int kind;  // PK: 0 below the tile's rows, 1 across the diagonal, 2 above (mirrored)
  };
  auto load = [&](Regs& R, int k0) {
    double* va = R.va;
    if constexpr (PK) {
      R.kind = k0 + 16 <= mu0 ? 0 : (k0 >= mu0 + 64 ? 2 : 1);
      if (R.kind == 0) {
        const double2 p0 = *reinterpret_cast<const double2*>(brow + k0 + lk);
        const double2 p1 = *reinterpret_cast<const double2*>(brow + k0 + lk + 2);
        va[0] = p0.x; va[1] = p0.y; va[2] = p1.x; va[3] = p1.y;
      } else if (R.kind == 2) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int nu = min(k0 + lkT + j, nao - 1);
          va[j] = bpk[(int64_t)nu * (nu + 1) / 2 + muT];
        }
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int nu = min(k0 + lk + j, nao - 1);
          va[j] = nu <= mu ? brow[nu] : bpk[(int64_t)nu * (nu + 1) / 2 + mu];
        }
      }
    } else if constexpr (VEC) {
      const double2 p0 = *reinterpret_cast<const double2*>(brow + k0 + lk);
      const double2 p1 = *reinterpret_cast<const double2*>(brow + k0 + lk + 2);
      va[0] = p0.x; va[1] = p0.y; va[2] = p1.x; va[3] = p1.y;
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int kk = k0 + lk + j;
        va[j] = (row_ok && kk < K) ? brow[kk] : 0.0;
      }
    }
#pragma unroll
    for (int j = 0; j < NF; ++j) {
      const int idx = t + 256 * j;
      const int kr = idx / NT, cc = idx - kr * NT;
      const int kk = k0 + kr, col = n0 + cc;
      R.vc[j] = (kk < K && col < nocc) ? C[(int64_t)kk * nocc + col] : 0.0;
    }
    // D values of the row dots (PK: not needed past the diagonal)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int kk = k0 + lk + j;
      R.vd[j] = (drow && row_ok && kk < K && !(PK && R.kind == 2)) ? drow[kk] : 0.0;
    }
  };
  // Screened B: only the 64-wide nu chunks that meet a kept block in some row
  // of this tile are visited, 16 k at a time.
  const unsigned long long live = cmask ? tile_chunks<1>(cmask, m0, M, nao, w, l) : 0ull;
  auto next_of = [&](int k) {
    if (k < 0) return -1;
    int kn = k + 16;
    if (cmask && kn % 64 == 0) {
      const int c = next_bit(live, k / 64);
      kn = c >= 0 ? 64 * c : -1;
    }
    return kn >= K ? -1 : kn;
  };
  int buf = 0;
  // one chunk: chunk k0 (in registers cur) into LDS stage buf, its row dots,
  // the barrier, the loads of the chunk after k1 (the one in flight in nx)
  // into cur, then the MFMAs of stage buf
  auto step = [&](Regs& cur, int& k0, int& k1) {
    if (PK && cur.kind == 2) {
#pragma unroll
      for (int j = 0; j < 4; ++j) As[buf][lrT][lkT + j] = k0 + lkT + j < nao ? cur.va[j] : 0.0;
    } else if (PK) {
#pragma unroll
      for (int j = 0; j < 4; ++j) As[buf][lr][lk + j] = k0 + lk + j < nao ? cur.va[j] : 0.0;
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) As[buf][lr][lk + j] = cur.va[j];
    }
#pragma unroll
    for (int j = 0; j < NF; ++j) {
      const int idx = t + 256 * j;
      const int kr = idx / NT, cc = idx - kr * NT;
      Cs[buf][kr][cc] = cur.vc[j];
    }
    if (drow && row_ok) {
      if constexpr (PK) {
        if (cur.kind != 2) {
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int kk = k0 + lk + j;
            const double wgt = kk < mu0 + lr ? 2.0 : (kk == mu0 + lr ? 1.0 : 0.0);
            rd = fma(cur.va[j] * wgt, cur.vd[j], rd);
          }
        }
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) rd = fma(cur.va[j], cur.vd[j], rd);
      }
    }
    __syncthreads();
    const int k2 = next_of(k1);
    if (k2 >= 0) load(cur, k2);
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const double a = As[buf][w * 16 + (l & 15)][kk * 4 + (l >> 4)];
#pragma unroll
      for (int f = 0; f < NF; ++f)
        acc[f] = mfma_f64(a, Cs[buf][kk * 4 + (l >> 4)][f * 16 + (l & 15)], acc[f]);
    }
    buf ^= 1;
    k0 = k1;
    k1 = k2;
  };
  Regs r0, r1;
  int k0 = cmask ? 64 * first_bit(live) : 0;
  if (k0 < 0 || k0 >= K) k0 = -1;
  int k1 = next_of(k0);
  if (k0 >= 0) load(r0, k0);
  if (k1 >= 0) load(r1, k1);
  while (k0 >= 0) {
    step(r0, k0, k1);
    if (k0 < 0) break;
    step(r1, k0, k1);
  }

  if (rowdot) {
    rd += __shfl_xor(rd, 1);
    rd += __shfl_xor(rd, 2);
    if ((t & 3) == 0 && row_ok && blockIdx.y == 0) rowdot[PK ? ptile * nao + mu0 + lr : grow] = rd;
  }

#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int64_t row = m0 + w * 16 + r * 4 + (l >> 4);
    const bool vr = PK ? mu0 + w * 16 + r * 4 + (l >> 4) < nao : row < M;
    const int64_t P = PK ? ptile : (vr ? row / nao : 0);
    const int mu_r = (int)(row - P * nao);
    const int64_t b = P / pblk;
    double* xrow = xlayout ? X + (((b * nao + mu_r) * pblk + (P - b * pblk)) * (int64_t)nocc)
                           : X + row * (int64_t)nocc;
    double rmax = 0.0;
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      const int col = n0 + f * 16 + (l & 15);
      if (vr && col < nocc) {
        const double z = acc[f][r];
        xrow[col] = z;
        rmax = fmax(rmax, fabs(z));
      }
    }
#pragma unroll
    for (int off = 1; off < 16; off <<= 1) rmax = fmax(rmax, __shfl_xor(rmax, off));
    if ((l & 15) == 0 && vr)
      atomicMax(&xmax[b * nao + mu_r], (unsigned long long)__double_as_longlong(rmax));
  }
}

__device__ __forceinline__ void lower_tile(int idx, int& t1, int& t2) {
  int r = (int)((sqrtf(8.0f * (float)idx + 1.0f) - 1.0f) * 0.5f);
  while ((r + 1) * (r + 2) / 2 <= idx) ++r;
  while (r * (r + 1) / 2 > idx) --r;
  t1 = r;
  t2 = idx - r * (r + 1) / 2;
}

// K partials (Eq. 6): Kp[grp][mu][nu] = sum over the aux blocks b of group grp
// of X_b X_b^T, with X_b rows contiguous (blocked layout, block stride
// pblk * nocc); lower 64x64 tiles, 4 waves of 32x32; 16 k at a time staged
// through LDS (double buffered, next chunk prefetched into registers).
__global__ __launch_bounds__(256) void k_k_fp64(const double* __restrict__ Xb, int64_t naux,
                                                int nao, int nocc, int pblk, int nb, int groups,
                                                double* __restrict__ Kp) {
  __shared__ double As[2][64][17];
  __shared__ double Bs[2][64][17];
  // group-major logical order, dealt to the XCDs in consecutive ranges (the
  // tiles of one group share X_b panels in one L2)
  const int64_t ntile = gridDim.x;
  const int64_t lid = xcd_order(blockIdx.x + (int64_t)blockIdx.y * ntile, ntile * gridDim.y);
  const int grp = (int)(lid / ntile);
  int t1, t2;
  lower_tile((int)(lid - grp * ntile), t1, t2);
  const int b_lo = (int)((int64_t)grp * nb / groups), b_hi = (int)((int64_t)(grp + 1) * nb / groups);
  const int t = threadIdx.x, w = t >> 6, l = t & 63;
  const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
  const int lr = t >> 2, li = (t & 3) * 4;
  const int mu_ld = t1 * 64 + lr, nu_ld = t2 * 64 + lr;
  const int64_t kfull = (int64_t)pblk * nocc;

  f64x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};

  // Two register sets of one 16-k chunk (4 values of row mu and of row nu per
  // thread): the loads of chunk c + 2 are issued while chunk c is multiplied.
  struct Regs {
    double va[4], vb[4];
  };
  auto kb_of = [&](int bb) {
    const int64_t p0 = (int64_t)bb * pblk;
    return (int)(((p0 + pblk < naux ? p0 + pblk : naux) - p0) * nocc);
  };
  auto load = [&](Regs& R, int b, int k0) {
    const int kb = kb_of(b);
    const double* xa = Xb + ((int64_t)b * nao + mu_ld) * kfull;
    const double* xb = Xb + ((int64_t)b * nao + nu_ld) * kfull;
    const int k = k0 + li;
    if (k + 4 <= kb && (kfull & 1) == 0) {  // 16-byte loads (rows start at even elements)
      if (mu_ld < nao) {
        const double2 p0 = *reinterpret_cast<const double2*>(xa + k);
        const double2 p1 = *reinterpret_cast<const double2*>(xa + k + 2);
        R.va[0] = p0.x; R.va[1] = p0.y; R.va[2] = p1.x; R.va[3] = p1.y;
      } else {
        R.va[0] = R.va[1] = R.va[2] = R.va[3] = 0.0;
      }
      if (nu_ld < nao) {
        const double2 p0 = *reinterpret_cast<const double2*>(xb + k);
        const double2 p1 = *reinterpret_cast<const double2*>(xb + k + 2);
        R.vb[0] = p0.x; R.vb[1] = p0.y; R.vb[2] = p1.x; R.vb[3] = p1.y;
      } else {
        R.vb[0] = R.vb[1] = R.vb[2] = R.vb[3] = 0.0;
      }
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        R.va[j] = (mu_ld < nao && k + j < kb) ? xa[k + j] : 0.0;
        R.vb[j] = (nu_ld < nao && k + j < kb) ? xb[k + j] : 0.0;
      }
    }
  };
  // flattened (block, k chunk) steps
  auto next_of = [&](int& b, int& k0) {
    if (b >= b_hi) return;
    k0 += 16;
    if (k0 >= kb_of(b)) {
      ++b;
      k0 = 0;
    }
  };
  int buf = 0;
  auto step = [&](Regs& cur, int& b, int& k0, int& b1, int& k1) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      As[buf][lr][li + j] = cur.va[j];
      Bs[buf][lr][li + j] = cur.vb[j];
    }
    __syncthreads();
    int b2 = b1, k2 = k1;
    next_of(b2, k2);
    if (b2 < b_hi) load(cur, b2, k2);
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const double a0 = As[buf][wr + (l & 15)][kk * 4 + (l >> 4)];
      const double a1 = As[buf][wr + 16 + (l & 15)][kk * 4 + (l >> 4)];
      const double b0 = Bs[buf][wc + (l & 15)][kk * 4 + (l >> 4)];
      const double b1v = Bs[buf][wc + 16 + (l & 15)][kk * 4 + (l >> 4)];
      acc[0][0] = mfma_f64(a0, b0, acc[0][0]);
      acc[0][1] = mfma_f64(a0, b1v, acc[0][1]);
      acc[1][0] = mfma_f64(a1, b0, acc[1][0]);
      acc[1][1] = mfma_f64(a1, b1v, acc[1][1]);
    }
    buf ^= 1;
    b = b1;
    k0 = k1;
    b1 = b2;
    k1 = k2;
  };
  Regs r0, r1;
  int b = b_lo, k0 = 0;
  int b1 = b, k1 = k0;
  next_of(b1, k1);
  if (b < b_hi) load(r0, b, k0);
  if (b1 < b_hi) load(r1, b1, k1);
  while (b < b_hi) {
    step(r0, b, k0, b1, k1);
    if (b >= b_hi) break;
    step(r1, b, k0, b1, k1);
  }

  double* out = Kp + (int64_t)grp * nao * nao;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int nu = t2 * 64 + wc + j * 16 + (l & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int mu = t1 * 64 + wr + i * 16 + r * 4 + (l >> 4);
        if (mu < nao && nu < nao) out[(int64_t)mu * nao + nu] = acc[i][j][r];
      }
    }
}

__global__ void k_xmax_to_exp(const unsigned long long* __restrict__ xmax, int64_t n,
                              int32_t* __restrict__ F) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    F[i] = exp_of_max(abs_max_bits_to_double(xmax[i]));
}

}  // namespace

template <bool PK, bool VEC>
static hipError_t launch_x_fp64_v(hipStream_t st, const double* B, int64_t naux, int nao,
                           const double* C, int nocc, double* X, int xlayout,
                           unsigned long long* xmax, int pblk, const double* D, double* rowdot,
                           const unsigned long long* cmask) {
  const int64_t M = naux * nao;
  const unsigned gx = PK ? (unsigned)(naux * ((nao + 63) / 64)) : (unsigned)((M + 63) / 64);
  if (nocc > 64) {
    hipLaunchKernelGGL((k_x_fp64<6, PK, VEC>), dim3(gx, (nocc + 95) / 96), dim3(256), 0, st, B, M,
                       nao, C, nocc, X, xlayout, xmax, nao, pblk, D, rowdot, cmask);
  } else if (nocc > 32) {
    hipLaunchKernelGGL((k_x_fp64<4, PK, VEC>), dim3(gx, 1), dim3(256), 0, st, B, M, nao, C, nocc,
                       X, xlayout, xmax, nao, pblk, D, rowdot, cmask);
  } else {
    hipLaunchKernelGGL((k_x_fp64<2, PK, VEC>), dim3(gx, 1), dim3(256), 0, st, B, M, nao, C, nocc,
                       X, xlayout, xmax, nao, pblk, D, rowdot, cmask);
  }
  return hipGetLastError();
}

hipError_t launch_x_fp64(hipStream_t st, const double* B, int64_t naux, int nao,
                         const double* C, int nocc, double* X, int xlayout,
                         unsigned long long* xmax, int pblk, const double* D, double* rowdot,
                         const unsigned long long* cmask, int packed) {
  if (naux * nao <= 0 || nocc <= 0) return hipSuccess;
  if (packed)
    return launch_x_fp64_v<true, false>(st, B, naux, nao, C, nocc, X, xlayout, xmax, pblk, D,
                                        rowdot, nullptr);
  if (nao % 16 == 0 && !cmask)
    return launch_x_fp64_v<false, true>(st, B, naux, nao, C, nocc, X, xlayout, xmax, pblk, D,
                                        rowdot, nullptr);
  return launch_x_fp64_v<false, false>(st, B, naux, nao, C, nocc, X, xlayout, xmax, pblk, D,
                                       rowdot, cmask);
}

hipError_t launch_k_fp64(hipStream_t st, const double* Xb, int64_t naux, int nao, int nocc,
                         int pblk, int nb, int groups, double* Kp) {
  const int nt = (nao + 63) / 64;
  hipLaunchKernelGGL(k_k_fp64, dim3((unsigned)(nt * (nt + 1) / 2), (unsigned)groups), dim3(256),
                     0, st, Xb, naux, nao, nocc, pblk, nb, groups, Kp);
  return hipGetLastError();
}

hipError_t launch_xmax_to_exp(hipStream_t st, const unsigned long long* xmax, int64_t n,
                              int32_t* F) {
  if (n <= 0) return hipSuccess;
  int64_t g = (n + 255) / 256;
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(k_xmax_to_exp, dim3((unsigned)g), dim3(256), 0, st, xmax, n, F);
  return hipGetLastError();
}

}  // namespace dfjk
