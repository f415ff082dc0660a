// Block screening of B (Sec. 2.1: shell pairs whose Schwarz estimate falls
// below a threshold are dropped, and B inherits that sparsity).  With shell
// blocks of `blk` consecutive basis functions, block (M, N) is dropped iff the
// Frobenius norm of B[:, M-block, N-block] over every aux index is below tau;
// the dropped entries are set to zero in B, so every consumer reads the same
// zeroed tensor, and the builds skip the 64-wide nu chunks that are zero.
#include "dfjk_internal.h"

namespace dfjk {
namespace {

// part[split][M][nu] = sum over P of the split and mu in shell row M of B^2.
__global__ __launch_bounds__(256) void k_shell_sq_partial(const double* __restrict__ B,
                                                          int64_t naux, int nao, int blk, int nsplit,
                                                          double* __restrict__ part) {
  const int M = blockIdx.x, split = blockIdx.y;
  const int64_t p_lo = (int64_t)split * naux / nsplit, p_hi = (int64_t)(split + 1) * naux / nsplit;
  const int mu0 = M * blk, mu1 = min(mu0 + blk, nao);
  const int64_t nn = (int64_t)nao * nao;
  for (int nu = threadIdx.x; nu < nao; nu += 256) {
    double a = 0.0;
    for (int64_t P = p_lo; P < p_hi; ++P)
      for (int mu = mu0; mu < mu1; ++mu) {
        const double v = B[P * nn + (int64_t)mu * nao + nu];
        a = fma(v, v, a);
      }
    part[((int64_t)split * gridDim.x + M) * nao + nu] = a;
  }
}

// norm(M, N) = sqrt(sum over splits, then over nu in shell column N); keep iff >= tau.
__global__ void k_shell_mask(const double* __restrict__ part, int nsplit, int nblk, int nao, int blk,
                             double tau, double* __restrict__ norms, uint8_t* __restrict__ mask) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)nblk * nblk) return;
  const int M = (int)(idx / nblk), N = (int)(idx - (int64_t)M * nblk);
  const int nu0 = N * blk, nu1 = min(nu0 + blk, nao);
  double s = 0.0;
  for (int sp = 0; sp < nsplit; ++sp) {
    const double* p = part + ((int64_t)sp * nblk + M) * nao;
    for (int nu = nu0; nu < nu1; ++nu) s += p[nu];
  }
  const double nrm = sqrt(s);
  if (norms) norms[idx] = nrm;
  mask[idx] = nrm >= tau ? 1 : 0;
}

// Zero the dropped blocks of B in place.
__global__ void k_apply_mask(double* __restrict__ B, int64_t naux, int nao, int blk, int nblk,
                             const uint8_t* __restrict__ mask) {
  const int64_t nn = (int64_t)nao * nao;
  const int64_t total = naux * nn;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e % nn;
    const int mu = (int)(r / nao), nu = (int)(r - (int64_t)mu * nao);
    if (!mask[(mu / blk) * nblk + nu / blk]) B[e] = 0.0;
  }
}

// chunks[mu] bit c: some kept block meets row mu in nu = 64 c .. 64 c + 63.
__global__ void k_chunk_bits(const uint8_t* __restrict__ mask, int nao, int blk, int nblk,
                             unsigned long long* __restrict__ chunks) {
  const int mu = blockIdx.x * blockDim.x + threadIdx.x;
  if (mu >= nao) return;
  const int M = mu / blk;
  unsigned long long bits = 0;
  for (int N = 0; N < nblk; ++N)
    if (mask[M * nblk + N]) {
      const int c0 = (N * blk) / 64, c1 = (min((N + 1) * blk, nao) - 1) / 64;
      for (int c = c0; c <= c1; ++c) bits |= 1ull << c;
    }
  chunks[mu] = bits;
}

inline unsigned gcap(int64_t n, int64_t c = 65536) {
  int64_t g = (n + 255) / 256;
  return (unsigned)(g < 1 ? 1 : (g > c ? c : g));
}

}  // namespace

hipError_t launch_screen(hipStream_t st, double* B, int64_t naux, int nao, int blk, double tau,
                         int nsplit, double* part, double* norms, uint8_t* mask,
                         unsigned long long* chunks) {
  const int nblk = (nao + blk - 1) / blk;
  hipLaunchKernelGGL(k_shell_sq_partial, dim3((unsigned)nblk, (unsigned)nsplit), dim3(256), 0, st, B,
                     naux, nao, blk, nsplit, part);
  hipLaunchKernelGGL(k_shell_mask, dim3(gcap((int64_t)nblk * nblk)), dim3(256), 0, st, part, nsplit,
                     nblk, nao, blk, tau, norms, mask);
  hipLaunchKernelGGL(k_apply_mask, dim3(gcap(naux * (int64_t)nao * nao)), dim3(256), 0, st, B, naux,
                     nao, blk, nblk, mask);
  hipLaunchKernelGGL(k_chunk_bits, dim3((unsigned)((nao + 255) / 256)), dim3(256), 0, st, mask, nao,
                     blk, nblk, chunks);
  return hipGetLastError();
}

}  // namespace dfjk
