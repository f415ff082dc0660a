// Peak probes of the device: the rates that the roofline fractions of the
// build are read against, measured on the device itself (INT8 MFMA loop,
// FP64 MFMA loop, streaming copy and streaming read of HBM).
#include "dfjk_internal.h"

namespace dfjk {
namespace {

// Each wave keeps CH independent accumulator chains (distinct operands) busy
// on one MFMA instruction; the operands stay in registers and this file is
// built with the accumulators in VGPRs, so the loop issues nothing but matrix
// instructions.  The sums are written out so that no chain is dead.
template <int CH>
__global__ __launch_bounds__(256) void k_peak_i8(int iters, int seed, int* __restrict__ out) {
  const int l = threadIdx.x;
  i32x4 a[CH], acc[CH];
#pragma unroll
  for (int c = 0; c < CH; ++c) {
    a[c] = i32x4{l * 0x01030507 + seed + c, (l ^ 0x5a5a5a5a) + 3 * c, seed * 0x0b0d0f11 - c, l + c};
    acc[c] = i32x4{c, -c, 2 * c, l};
  }
  const i32x4 b = {seed ^ 0x13171d1f, l * 0x1f1d1713, 0x7f7f7f7f - l, seed};
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < CH; ++c) acc[c] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[c], b, acc[c], 0, 0, 0);
  }
  int sum = 0;
#pragma unroll
  for (int c = 0; c < CH; ++c) sum += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  out[(int64_t)blockIdx.x * blockDim.x + l] = sum;
}

template <int CH>
__global__ __launch_bounds__(256) void k_peak_f64(int iters, int seed, double* __restrict__ out) {
  const int l = threadIdx.x;
  double a[CH];
  f64x4 acc[CH];
#pragma unroll
  for (int c = 0; c < CH; ++c) {
    a[c] = 1.0 + 0x1p-20 * (l + seed + c);
    acc[c] = f64x4{(double)c, (double)l, 0.0, -1.0 * c};
  }
  const double b = 1.0 - 0x1p-21 * l;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < CH; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[c], b, acc[c], 0, 0, 0);
  }
  double sum = 0.0;
#pragma unroll
  for (int c = 0; c < CH; ++c) sum += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  out[(int64_t)blockIdx.x * blockDim.x + l] = sum;
}

// Streaming copy: 16-byte loads and stores, four in flight per thread.
__global__ __launch_bounds__(256) void k_peak_copy(const int4* __restrict__ src,
                                                   int4* __restrict__ dst, int64_t n16) {
  const int64_t stride = (int64_t)gridDim.x * 256;
  int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  for (; i + 3 * stride < n16; i += 4 * stride) {
    const int4 v0 = src[i], v1 = src[i + stride], v2 = src[i + 2 * stride], v3 = src[i + 3 * stride];
    dst[i] = v0;
    dst[i + stride] = v1;
    dst[i + 2 * stride] = v2;
    dst[i + 3 * stride] = v3;
  }
  for (; i < n16; i += stride) dst[i] = src[i];
}

// Streaming read: 16-byte loads, eight in flight per thread, one word written
// per thread.
__global__ __launch_bounds__(256) void k_peak_read(const int4* __restrict__ src, int64_t n16,
                                                   int* __restrict__ out) {
  const int64_t stride = (int64_t)gridDim.x * 256;
  int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  int acc = 0;
  for (; i + 7 * stride < n16; i += 8 * stride) {
    int4 v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = src[i + u * stride];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc ^= v[u].x ^ v[u].w;
  }
  for (; i < n16; i += stride) acc ^= src[i].x;
  out[(int64_t)blockIdx.x * 256 + threadIdx.x] = acc;
}

}  // namespace

hipError_t launch_peak(hipStream_t st, int kind, int ncu, void* buf, size_t bytes, int iters,
                       double* work) {
  constexpr int kCh = 8;
  if (kind == 0 || kind == 1) {
    const unsigned grid = (unsigned)ncu * 8;  // 32 waves per CU
    if (bytes < (size_t)grid * 256 * 8) return hipErrorInvalidValue;
    if (kind == 0) {
      hipLaunchKernelGGL(k_peak_i8<kCh>, dim3(grid), dim3(256), 0, st, iters, 3,
                         reinterpret_cast<int*>(buf));
      *work = (double)grid * 4 * iters * kCh * (16.0 * 16 * 64 * 2);
    } else {
      hipLaunchKernelGGL(k_peak_f64<kCh>, dim3(grid), dim3(256), 0, st, iters, 3,
                         reinterpret_cast<double*>(buf));
      *work = (double)grid * 4 * iters * kCh * (16.0 * 16 * 4 * 2);
    }
    return hipGetLastError();
  }
  const unsigned grid = (unsigned)ncu * 8;
  if (kind == 2) {
    const int64_t n16 = (int64_t)(bytes / 2 / 16);
    if (n16 < 1) return hipErrorInvalidValue;
    const int4* src = reinterpret_cast<const int4*>(buf);
    int4* dst = reinterpret_cast<int4*>(buf) + n16;
    hipLaunchKernelGGL(k_peak_copy, dim3(grid), dim3(256), 0, st, src, dst, n16);
    *work = 2.0 * 16.0 * (double)n16;
    return hipGetLastError();
  }
  if (kind == 3) {
    const size_t outb = (size_t)grid * 256 * 4;
    if (bytes < outb + 16 * 1024) return hipErrorInvalidValue;
    const int64_t n16 = (int64_t)((bytes - outb) / 16);
    int* out = reinterpret_cast<int*>(reinterpret_cast<char*>(buf) + (size_t)n16 * 16);
    hipLaunchKernelGGL(k_peak_read, dim3(grid), dim3(256), 0, st,
                       reinterpret_cast<const int4*>(buf), n16, out);
    *work = 16.0 * (double)n16;
    return hipGetLastError();
  }
  return hipErrorInvalidValue;
}

}  // namespace dfjk
