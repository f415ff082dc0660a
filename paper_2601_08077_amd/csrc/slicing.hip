// Exponents and INT8 digit planes of FP64 operands (Sec. 3.2: s INT8 splits per
// input; per-row power-of-two scaling).  gfx950.
#include "dfjk_internal.h"

namespace dfjk {
namespace {

// One wavefront per row: e[r] = exponent of max_c |A[r][c]|; NaN/Inf -> status.
__global__ __launch_bounds__(256) void k_row_exp(const double* __restrict__ A, int64_t rows,
                                                 int64_t cols, int64_t lda,
                                                 int32_t* __restrict__ e, int* status) {
  const int lane = threadIdx.x & 63;
  const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t r = wid; r < rows; r += nw) {
    const double* a = A + r * lda;
    double m = 0.0;
    bool bad = false;
    for (int64_t c = lane; c < cols; c += kWave) {
      const double v = a[c];
      bad |= !isfinite(v);
      m = fmax(m, fabs(v));
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) m = fmax(m, __shfl_xor(m, off));
    if (__any(bad) && lane == 0) atomicOr(status, kStatusNonFinite);
    if (lane == 0) e[r] = exp_of_max(m);
  }
}

// Row exponents of packed B (B_P stored as its lower triangle by rows, element
// (mu, nu), mu >= nu, at mu (mu + 1) / 2 + nu): the maximum of row mu of B_P
// is the maximum over its stored row (nu <= mu) and over column mu of the rows
// below (nu > mu).  Workgroup (64 rows, P): waves take rows for the first part
// (lanes along the row), lanes take the 64 rows for the second (each load
// instruction reads 64 consecutive mu of one stored row nu).
__global__ __launch_bounds__(256) void k_row_exp_packed(const double* __restrict__ B, int nao,
                                                        int32_t* __restrict__ e, int* status) {
  __shared__ double rowm[64];
  __shared__ double part[4][64];
  const int t = threadIdx.x, w = t >> 6, l = t & 63;
  const int mu0 = blockIdx.x * 64;
  const int64_t P = blockIdx.y;
  const double* bp = B + P * ((int64_t)nao * (nao + 1) / 2);
  bool bad = false;
  for (int r = w; r < 64; r += 4) {
    const int mu = mu0 + r;
    double m = 0.0;
    if (mu < nao) {
      const double* row = bp + (int64_t)mu * (mu + 1) / 2;
      for (int nu = l; nu <= mu; nu += kWave) {
        const double v = row[nu];
        bad |= !isfinite(v);
        m = fmax(m, fabs(v));
      }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) m = fmax(m, __shfl_xor(m, off));
    if (l == 0) rowm[r] = m;
  }
  const int mu = mu0 + l;
  double m2 = 0.0;
  if (mu < nao) {
    for (int nu = mu0 + 1 + w; nu < nao; nu += 4) {
      if (nu > mu) {
        const double v = bp[(int64_t)nu * (nu + 1) / 2 + mu];
        bad |= !isfinite(v);
        m2 = fmax(m2, fabs(v));
      }
    }
  }
  part[w][l] = m2;
  if (__any(bad) && l == 0) atomicOr(status, kStatusNonFinite);
  __syncthreads();
  if (w == 0 && mu < nao) {
    const double m = fmax(fmax(rowm[l], part[0][l]), fmax(fmax(part[1][l], part[2][l]), part[3][l]));
    e[P * nao + mu] = exp_of_max(m);
  }
}

// f[i] = exponent of max_nu |C[nu][i]| (the columns of C are the rows of the
// right operand of Eq. 5 over its contraction index nu): one wavefront per column.
__global__ __launch_bounds__(256) void k_col_exp(const double* __restrict__ C, int64_t nao,
                                                 int64_t nocc, int32_t* __restrict__ f,
                                                 int* status) {
  const int lane = threadIdx.x & 63;
  const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (i >= nocc) return;
  double m = 0.0;
  bool bad = false;
  for (int64_t k = lane; k < nao; k += kWave) {
    const double v = C[k * nocc + i];
    bad |= !isfinite(v);
    m = fmax(m, fabs(v));
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) m = fmax(m, __shfl_xor(m, off));
  if (__any(bad) && lane == 0) atomicOr(status, kStatusNonFinite);
  if (lane == 0) f[i] = exp_of_max(m);
}

// digits[a][r][c] for a = 0..s-1 (a = 0 is d_1).
__global__ void k_slice_rows(const double* __restrict__ A, int64_t rows, int64_t cols,
                             int64_t lda, int s, const int32_t* __restrict__ e,
                             int8_t* __restrict__ digits) {
  const int64_t n = rows * cols;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = idx / cols, c = idx - r * cols;
    const uint64_t w = digit_word(A[r * lda + c], e[r]);
    for (int a = 0; a < s; ++a) digits[(int64_t)a * n + idx] = (int8_t)digit_byte(w, a + 1);
  }
}

// Digit planes of C^T in the right-operand layout of the INT8 X product,
// tiled by 64-wide k chunks: plane a, chunk c, column i holds 64 bytes at
// a ncp kp + (c ncp + i) 64, byte p = 16 q + 8 b + 2 j + h holding
// k = 64 c + 16 j + 4 q + 2 b + h (the order in which the B-tile loader's
// eight lanes per row place their values in the four MFMA lane groups).
// With `natural` set: dC[a][i][k] in natural order (X from B digit planes).
__global__ void k_slice_c(const double* __restrict__ C, int64_t nao, int64_t nocc, int s,
                          const int32_t* __restrict__ f, int ncp, int kp, int natural,
                          int8_t* __restrict__ dC) {
  const int64_t n = (int64_t)ncp * kp;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(idx / kp);
    const int p = (int)(idx - (int64_t)i * kp);
    const int c = p >> 6, q = (p >> 4) & 3, b = (p >> 3) & 1, j = (p >> 1) & 3, h = p & 1;
    const int64_t k = natural ? p : (int64_t)c * 64 + 16 * j + 4 * q + 2 * b + h;
    const int64_t o = natural ? idx : ((int64_t)c * ncp + i) * 64 + (p & 63);
    uint64_t w = 0;
    if (i < nocc && k < nao) w = digit_word(C[k * nocc + i], f[i]);
    for (int a = 0; a < s; ++a) dC[(int64_t)a * n + o] = (int8_t)digit_byte(w, a + 1);
  }
}

__global__ void k_fill_u64(unsigned long long* p, int64_t n, unsigned long long v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_fill_i32(int* p, int64_t n, int v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

inline unsigned grid_for(int64_t n, int block, int64_t cap = 65536) {
  int64_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

}  // namespace

hipError_t launch_row_exp(hipStream_t st, const double* A, int64_t rows, int64_t cols,
                          int64_t lda, int32_t* e, int* status) {
  if (rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_row_exp, dim3(grid_for(rows * 64, 256)), dim3(256), 0, st, A, rows,
                     cols, lda, e, status);
  return hipGetLastError();
}

hipError_t launch_row_exp_packed(hipStream_t st, const double* B, int64_t naux, int nao,
                                 int32_t* e, int* status) {
  if (naux <= 0 || nao <= 0) return hipSuccess;
  const dim3 grid((unsigned)((nao + 63) / 64), (unsigned)naux);
  hipLaunchKernelGGL(k_row_exp_packed, grid, dim3(256), 0, st, B, nao, e, status);
  return hipGetLastError();
}

hipError_t launch_col_exp(hipStream_t st, const double* C, int64_t nao, int64_t nocc,
                          int32_t* f, int* status) {
  if (nocc <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_col_exp, dim3(grid_for(nocc * 64, 256)), dim3(256), 0, st, C, nao, nocc, f,
                     status);
  return hipGetLastError();
}

hipError_t launch_slice_rows(hipStream_t st, const double* A, int64_t rows, int64_t cols,
                             int64_t lda, int s, const int32_t* e, int8_t* digits) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_slice_rows, dim3(grid_for(rows * cols, 256)), dim3(256), 0, st, A,
                     rows, cols, lda, s, e, digits);
  return hipGetLastError();
}

hipError_t launch_slice_c(hipStream_t st, const double* C, int64_t nao, int64_t nocc, int s,
                          const int32_t* f, int ncp, int kp, int natural, int8_t* dC) {
  hipLaunchKernelGGL(k_slice_c, dim3(grid_for((int64_t)ncp * kp, 256)), dim3(256), 0, st, C,
                     nao, nocc, s, f, ncp, kp, natural, dC);
  return hipGetLastError();
}

hipError_t launch_fill_u64(hipStream_t st, unsigned long long* p, int64_t n,
                           unsigned long long v) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(n, 256, 4096)), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

hipError_t launch_fill_i32(hipStream_t st, int* p, int64_t n, int v) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n, 256, 4096)), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

}  // namespace dfjk
