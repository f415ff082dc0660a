// Metric Cholesky and whitening of the three-index tensor (Sec. 2.1, Eq. 2):
// W = L L^T, then B = L^-1 T over the aux index.  FP64 throughout (the metric
// Cholesky is one of the places where FP64 stays on the GPU).  Blocked
// right-looking algorithms with 64-wide blocks; the bulk of the work (trailing
// updates, the triangular inverse's updates and the whitening product) runs on
// one FP64-MFMA GEMM kernel (v_mfma_f64_16x16x4_f64).
#include "dfjk_internal.h"

namespace dfjk {
namespace {

__device__ __forceinline__ f64x4 mfma_f64(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// C = alpha op(A) op(B) + beta C on 64x64 tiles, 4 waves of 32x32.
//   A [M][K] (lda); B [K][N] (ldb) or, with TRANSB, B [N][K] (ldb);
//   LOWER_A: A is lower triangular, so row tile r only needs k < 64 (r + 1);
//   LOWER_C: only tiles with col0 <= row0 are computed (symmetric updates).
// beta == 0 does not read C.  Grid: x = row tiles, y = column tiles, so that
// the workgroups running together share a column panel of B.
template <bool TRANSB, bool LOWER_A, bool LOWER_C>
__global__ __launch_bounds__(256) void k_gemm_f64(int64_t M, int64_t N, int64_t K, double alpha,
                                                  const double* __restrict__ A, int64_t lda,
                                                  const double* __restrict__ Bm, int64_t ldb,
                                                  double beta, double* __restrict__ C,
                                                  int64_t ldc) {
  __shared__ double As[2][64][17];
  __shared__ double Bs[2][16][65];
  const int64_t row0 = (int64_t)blockIdx.x * 64, col0 = (int64_t)blockIdx.y * 64;
  if (LOWER_C && col0 > row0) return;
  const int t = threadIdx.x, w = t >> 6, l = t & 63;
  const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
  int64_t kmax = K;
  if (LOWER_A && row0 + 64 < kmax) kmax = row0 + 64;

  f64x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};

  double va[4], vb[4];
  const int ar = t >> 2, ak = (t & 3) * 4;  // A tile loader: row, 4 consecutive k
  // B loader: NN: k = t / 16, 4 consecutive n; TRANSB: n = t / 4, 4 consecutive k
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t r = row0 + ar, k = k0 + ak + j;
      va[j] = (r < M && k < kmax) ? A[r * lda + k] : 0.0;
    }
    if (!TRANSB) {
      const int bk = t >> 4, bn = (t & 15) * 4;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int64_t k = k0 + bk, n = col0 + bn + j;
        vb[j] = (k < kmax && n < N) ? Bm[k * ldb + n] : 0.0;
      }
    } else {
      const int bn = t >> 2, bk = (t & 3) * 4;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int64_t k = k0 + bk + j, n = col0 + bn;
        vb[j] = (k < kmax && n < N) ? Bm[n * ldb + k] : 0.0;
      }
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int j = 0; j < 4; ++j) As[buf][ar][ak + j] = va[j];
    if (!TRANSB) {
      const int bk = t >> 4, bn = (t & 15) * 4;
#pragma unroll
      for (int j = 0; j < 4; ++j) Bs[buf][bk][bn + j] = vb[j];
    } else {
      const int bn = t >> 2, bk = (t & 3) * 4;
#pragma unroll
      for (int j = 0; j < 4; ++j) Bs[buf][bk + j][bn] = vb[j];
    }
  };

  int buf = 0;
  if (kmax > 0) load(0);
  for (int64_t k0 = 0; k0 < kmax; k0 += 16, buf ^= 1) {
    store(buf);
    __syncthreads();
    if (k0 + 16 < kmax) load(k0 + 16);
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const double a0 = As[buf][wr + (l & 15)][kk * 4 + (l >> 4)];
      const double a1 = As[buf][wr + 16 + (l & 15)][kk * 4 + (l >> 4)];
      const double b0 = Bs[buf][kk * 4 + (l >> 4)][wc + (l & 15)];
      const double b1 = Bs[buf][kk * 4 + (l >> 4)][wc + 16 + (l & 15)];
      acc[0][0] = mfma_f64(a0, b0, acc[0][0]);
      acc[0][1] = mfma_f64(a0, b1, acc[0][1]);
      acc[1][0] = mfma_f64(a1, b0, acc[1][0]);
      acc[1][1] = mfma_f64(a1, b1, acc[1][1]);
    }
  }

#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int64_t c = col0 + wc + j * 16 + (l & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = row0 + wr + i * 16 + r * 4 + (l >> 4);
        if (row < M && c < N) {
          double v = alpha * acc[i][j][r];
          if (beta != 0.0) v = fma(beta, C[row * ldc + c], v);
          C[row * ldc + c] = v;
        }
      }
    }
}

// Unblocked Cholesky of the kb x kb diagonal block at A (lower part), in LDS.
// A non-positive pivot sets the status word and leaves NaN in the block.
__global__ __launch_bounds__(256) void k_potrf_diag(double* __restrict__ A, int64_t lda, int kb,
                                                    int* status) {
  __shared__ double S[64][65];
  const int t = threadIdx.x;
  for (int e = t; e < kb * kb; e += 256) {
    const int i = e / kb, j = e - i * kb;
    S[i][j] = j <= i ? A[i * lda + j] : 0.0;
  }
  __syncthreads();
  for (int j = 0; j < kb; ++j) {
    if (t == 0) {
      const double d = S[j][j];
      if (!(d > 0.0)) atomicOr(status, kStatusNotSpd);
      S[j][j] = sqrt(d);
    }
    __syncthreads();
    const double d = S[j][j];
    for (int i = j + 1 + t; i < kb; i += 256) S[i][j] /= d;
    __syncthreads();
    // trailing update of the lower triangle: S[i][m] -= S[i][j] S[m][j], j < m <= i
    const int rem = kb - j - 1;
    for (int e = t; e < rem * rem; e += 256) {
      const int i = j + 1 + e / rem, m = j + 1 + e % rem;
      if (m <= i) S[i][m] -= S[i][j] * S[m][j];
    }
    __syncthreads();
  }
  for (int e = t; e < kb * kb; e += 256) {
    const int i = e / kb, j = e - i * kb;
    if (j <= i) A[i * lda + j] = S[i][j];
  }
}

// Panel below a factored diagonal block: row i of P (kb wide) <- P_i L_kk^-T,
// i.e. forward substitution x_j = (p_j - sum_{m<j} x_m L_jm) / L_jj.
// One thread per row; the factored block and the rows live in LDS.
__global__ __launch_bounds__(64) void k_trsm_panel(const double* __restrict__ Lkk, int64_t lda,
                                                   double* __restrict__ Pn, int64_t rows, int kb) {
  __shared__ double Ls[64][65];
  __shared__ double X[64][65];  // X[j][thread]
  const int t = threadIdx.x;
  for (int e = t; e < kb * kb; e += 64) {
    const int i = e / kb, j = e - i * kb;
    Ls[i][j] = Lkk[i * lda + j];
  }
  const int64_t r = (int64_t)blockIdx.x * 64 + t;
  const bool ok = r < rows;
  for (int j = 0; j < kb; ++j) X[j][t] = ok ? Pn[r * lda + j] : 0.0;
  __syncthreads();
  for (int j = 0; j < kb; ++j) {
    double x = X[j][t];
    for (int m = 0; m < j; ++m) x -= X[m][t] * Ls[j][m];
    X[j][t] = x / Ls[j][j];
  }
  if (ok)
    for (int j = 0; j < kb; ++j) Pn[r * lda + j] = X[j][t];
}

// Rows i0 .. i0 + ib of R (ncols columns) <- L_ii^-1 R_i (forward substitution
// per column, one thread per column).
__global__ __launch_bounds__(64) void k_trsm_left_diag(const double* __restrict__ Lii, int64_t ldl,
                                                       double* __restrict__ R, int64_t ldr,
                                                       int ib, int64_t ncols) {
  __shared__ double Ls[64][65];
  const int t = threadIdx.x;
  for (int e = t; e < ib * ib; e += 64) {
    const int i = e / ib, j = e - i * ib;
    Ls[i][j] = Lii[i * ldl + j];
  }
  __syncthreads();
  const int64_t c = (int64_t)blockIdx.x * 64 + t;
  if (c >= ncols) return;
  double x[64];
#pragma unroll
  for (int j = 0; j < 64; ++j) x[j] = j < ib ? R[j * ldr + c] : 0.0;
#pragma unroll
  for (int j = 0; j < 64; ++j) {
    if (j < ib) {
      double v = x[j];
#pragma unroll
      for (int m = 0; m < j; ++m) v -= Ls[j][m] * x[m];
      x[j] = v / Ls[j][j];
    }
  }
#pragma unroll
  for (int j = 0; j < 64; ++j)
    if (j < ib) R[j * ldr + c] = x[j];
}

__global__ void k_identity(double* __restrict__ A, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * n;
       e += (int64_t)gridDim.x * blockDim.x)
    A[e] = (e / n == e % n) ? 1.0 : 0.0;
}

__global__ void k_zero_upper(double* __restrict__ A, int64_t n, int64_t lda) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / n, j = e % n;
    if (j > i) A[i * lda + j] = 0.0;
  }
}

inline unsigned cap_grid(int64_t n, int64_t cap = 4096) {
  int64_t g = (n + 255) / 256;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

template <bool TB, bool LA, bool LC>
hipError_t gemm(hipStream_t st, int64_t M, int64_t N, int64_t K, double alpha, const double* A,
                int64_t lda, const double* Bm, int64_t ldb, double beta, double* C, int64_t ldc) {
  if (M <= 0 || N <= 0) return hipSuccess;
  const int64_t gy = (N + 63) / 64;
  for (int64_t y0 = 0; y0 < gy; y0 += 65535) {  // grid y limit
    const int64_t ny = gy - y0 < 65535 ? gy - y0 : 65535;
    hipLaunchKernelGGL((k_gemm_f64<TB, LA, LC>), dim3((unsigned)((M + 63) / 64), (unsigned)ny),
                       dim3(256), 0, st, M, N - y0 * 64, K, alpha, A, lda, Bm + (TB ? y0 * 64 * ldb : y0 * 64),
                       ldb, beta, C + y0 * 64, ldc);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_cholesky(hipStream_t st, double* A, int64_t n, int* status) {
  for (int64_t k0 = 0; k0 < n; k0 += 64) {
    const int kb = (int)(n - k0 < 64 ? n - k0 : 64);
    hipLaunchKernelGGL(k_potrf_diag, dim3(1), dim3(256), 0, st, A + k0 * n + k0, n, kb, status);
    const int64_t rest = n - k0 - kb;
    if (rest > 0) {
      double* P = A + (k0 + kb) * n + k0;
      hipLaunchKernelGGL(k_trsm_panel, dim3((unsigned)((rest + 63) / 64)), dim3(64), 0, st,
                         A + k0 * n + k0, n, P, rest, kb);
      const hipError_t e = gemm<true, false, true>(st, rest, rest, kb, -1.0, P, n, P, n, 1.0,
                                                   A + (k0 + kb) * n + k0 + kb, n);
      if (e != hipSuccess) return e;
    }
  }
  hipLaunchKernelGGL(k_zero_upper, dim3(cap_grid(n * n)), dim3(256), 0, st, A, n, n);
  return hipGetLastError();
}

hipError_t launch_tri_inverse(hipStream_t st, const double* L, int64_t n, double* Linv) {
  hipLaunchKernelGGL(k_identity, dim3(cap_grid(n * n)), dim3(256), 0, st, Linv, n);
  for (int64_t i0 = 0; i0 < n; i0 += 64) {
    const int ib = (int)(n - i0 < 64 ? n - i0 : 64);
    const int64_t ncols = i0 + ib;  // columns of rows i0.. that can be nonzero
    hipLaunchKernelGGL(k_trsm_left_diag, dim3((unsigned)((ncols + 63) / 64)), dim3(64), 0, st,
                       L + i0 * n + i0, n, Linv + i0 * n, n, ib, ncols);
    const int64_t rest = n - i0 - ib;
    if (rest > 0) {
      const hipError_t e = gemm<false, false, false>(st, rest, ncols, ib, -1.0, L + (i0 + ib) * n + i0,
                                                     n, Linv + i0 * n, n, 1.0, Linv + (i0 + ib) * n, n);
      if (e != hipSuccess) return e;
    }
  }
  return hipGetLastError();
}

hipError_t launch_density(hipStream_t st, const double* C, int64_t nao, int64_t nocc, double occ,
                          double* D) {
  return gemm<true, false, false>(st, nao, nao, nocc, occ, C, nocc, C, nocc, 0.0, D, nao);
}

hipError_t launch_whiten(hipStream_t st, const double* Linv, int64_t naux, const double* T,
                         int64_t ncols, double* Bout) {
  return gemm<false, true, false>(st, naux, ncols, naux, 1.0, Linv, naux, T, ncols, 0.0, Bout, ncols);
}

}  // namespace dfjk
