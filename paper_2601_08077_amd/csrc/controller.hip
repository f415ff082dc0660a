// Learned slice controller: the per-block statistics that feed it, its
// 16 -> 64 -> 64 -> 8 perceptron (FP32: forward, backward, Adam), the slice
// choice and the FP64 check of emulated block partials.  The controller
// extends the per-iteration precision rule (Sec. 3.2, Eq. 11, Table 1) to one
// slice count per aux block, following the outlook of Sec. 5.
#include "dfjk_internal.h"

namespace dfjk {
namespace {

constexpr int NI = 16, NH = 64, NO = 8;
constexpr int OW1 = 0, OB1 = OW1 + NI * NH, OW2 = OB1 + NH, OB2 = OW2 + NH * NH, OW3 = OB2 + NH,
              OB3 = OW3 + NH * NO, NPARAM = OB3 + NO;
constexpr int MT = 32;  // samples per workgroup

// ---------------------------------------------------------------- statistics
// Block statistics of X recorded by the build itself: out[b] = (max over mu of
// xmax[b][mu] (bit patterns of non-negative doubles), the sum of the block's
// nslot squared-sum slots, lane-strided then a fixed shuffle tree).  One wave
// per block.
__global__ __launch_bounds__(64) void k_xstats_from(const unsigned long long* __restrict__ xmax,
                                                    const double* __restrict__ xss, int nao,
                                                    int64_t nslot, double* __restrict__ out) {
  const int b = blockIdx.x, l = threadIdx.x;
  unsigned long long m = 0;
  for (int mu = l; mu < nao; mu += 64) {
    const unsigned long long v = xmax[(int64_t)b * nao + mu];
    m = v > m ? v : m;
  }
  double sq = 0.0;
  for (int64_t i = l; i < nslot; i += 64) sq += xss[b * nslot + i];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const unsigned long long o = __shfl_xor(m, off);
    m = o > m ? o : m;
    sq += __shfl_xor(sq, off);
  }
  if (l == 0) {
    out[2 * b] = abs_max_bits_to_double(m);
    out[2 * b + 1] = sq;
  }
}

// partial[seg][split] = (max |a - a2|, sum (a - a2)^2) over the split's slice of
// segment seg (segments of seglen elements, the last one ragged).  In the last
// segment only the first last_valid elements of every run of rowlen count
// (the ragged last aux block of the blocked X layout).
__global__ __launch_bounds__(256) void k_seg_stats_partial(const double* __restrict__ A,
                                                           const double* __restrict__ A2,
                                                           int64_t n, int64_t seglen, int64_t rowlen,
                                                           int64_t last_valid, int nsplit,
                                                           double* __restrict__ partial) {
  __shared__ double red[2][4];
  const int64_t seg = blockIdx.x;
  const int split = blockIdx.y;
  const int64_t s0 = seg * seglen;
  const int64_t len = (s0 + seglen < n ? s0 + seglen : n) - s0;
  const int64_t a = s0 + split * len / nsplit, b = s0 + (split + 1) * len / nsplit;
  const bool last = seg == (int64_t)gridDim.x - 1 && last_valid < rowlen;
  double m = 0.0, ss = 0.0;
  for (int64_t i = a + threadIdx.x; i < b; i += 256) {
    if (last && (i - s0) % rowlen >= last_valid) continue;
    const double v = A2 ? A[i] - A2[i] : A[i];
    m = fmax(m, fabs(v));
    ss = fma(v, v, ss);
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    m = fmax(m, __shfl_xor(m, off));
    ss += __shfl_xor(ss, off);
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = m;
    red[1][threadIdx.x >> 6] = ss;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double* o = partial + 2 * (seg * nsplit + split);
    o[0] = fmax(fmax(red[0][0], red[0][1]), fmax(red[0][2], red[0][3]));
    o[1] = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
  }
}

__global__ void k_seg_stats_final(const double* __restrict__ partial, int64_t nseg, int nsplit,
                                  double* __restrict__ out) {
  const int64_t seg = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (seg >= nseg) return;
  double m = 0.0, ss = 0.0;
  for (int k = 0; k < nsplit; ++k) {
    m = fmax(m, partial[2 * (seg * nsplit + k)]);
    ss += partial[2 * (seg * nsplit + k) + 1];
  }
  out[2 * seg] = m;
  out[2 * seg + 1] = ss;
}

__device__ __forceinline__ float log2_or(double v) { return v > 0.0 ? (float)log2(v) : -1100.0f; }
__device__ __forceinline__ float log10_or(double v) { return v > 0.0 ? (float)log10(v) : -330.0f; }

// Features of every block (row b of feat[nb][16]).
__global__ void k_features(const double* __restrict__ bstats, const double* __restrict__ xstats,
                           const double* __restrict__ dstat, const double* __restrict__ cstat,
                           const double* __restrict__ kstat, CtlScalars sc, int nb,
                           float* __restrict__ feat) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  float* f = feat + (int64_t)b * NI;
  f[0] = log2_or(bstats[2 * b]);
  f[1] = log2_or(sqrt(bstats[2 * b + 1]));
  f[2] = log10_or(sqrt(dstat[1]));
  f[3] = (float)(sc.iteration / sc.n_iter);
  f[4] = log10_or(sc.de_rel);
  f[5] = log2_or(cstat[0]);
  f[6] = log2_or(xstats[2 * b]);
  f[7] = log2_or(sqrt(xstats[2 * b + 1]));
  f[8] = log2_or(sqrt(kstat[1]));
  f[9] = log10_or(sc.target);
  f[10] = (float)log2(sc.nao);
  f[11] = (float)log2(sc.naux);
  f[12] = (float)log2(sc.nocc);
  f[13] = (float)(sc.plain_s / 8.0);
  f[14] = (float)((double)b / nb);
  f[15] = 1.0f;
}

// ------------------------------------------------------------------ perceptron
// Parameters W1[16][64] b1[64] W2[64][64] b2[64] W3[64][8] b3[8] (row-major).
struct MlpLds {
  float w[NPARAM];
  float x[MT][NI];
  float z1[MT][NH];
  float z2[MT][NH];
  float dy[MT][NO];
};

__device__ void mlp_load(MlpLds& L, const float* __restrict__ prm, const float* __restrict__ x,
                         const int32_t* __restrict__ idx, int64_t n, int64_t r0) {
  for (int i = threadIdx.x; i < NPARAM; i += 256) L.w[i] = prm[i];
  for (int i = threadIdx.x; i < MT * NI; i += 256) {
    const int r = i / NI, c = i - r * NI;
    const int64_t row = r0 + r;
    float v = 0.0f;
    if (row < n) v = x[(idx ? (int64_t)idx[row] : row) * NI + c];
    L.x[r][c] = v;
  }
  __syncthreads();
}

// z1 = x W1 + b1, z2 = relu(z1) W2 + b2 (fixed k order), y = relu(z2) W3 + b3.
__device__ void mlp_forward(MlpLds& L, float (*y)[NO]) {
  for (int i = threadIdx.x; i < MT * NH; i += 256) {
    const int r = i / NH, c = i - r * NH;
    float a = L.w[OB1 + c];
    for (int k = 0; k < NI; ++k) a = fmaf(L.x[r][k], L.w[OW1 + k * NH + c], a);
    L.z1[r][c] = a;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < MT * NH; i += 256) {
    const int r = i / NH, c = i - r * NH;
    float a = L.w[OB2 + c];
    for (int k = 0; k < NH; ++k) a = fmaf(fmaxf(L.z1[r][k], 0.0f), L.w[OW2 + k * NH + c], a);
    L.z2[r][c] = a;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < MT * NO; i += 256) {
    const int r = i / NO, c = i - r * NO;
    float a = L.w[OB3 + c];
    for (int k = 0; k < NH; ++k) a = fmaf(fmaxf(L.z2[r][k], 0.0f), L.w[OW3 + k * NO + c], a);
    y[r][c] = a;
  }
  __syncthreads();
}

__global__ __launch_bounds__(256) void k_mlp_forward(const float* __restrict__ prm,
                                                     const float* __restrict__ x, int64_t n,
                                                     float* __restrict__ y) {
  __shared__ MlpLds L;
  const int64_t r0 = (int64_t)blockIdx.x * MT;
  mlp_load(L, prm, x, nullptr, n, r0);
  mlp_forward(L, L.dy);
  for (int i = threadIdx.x; i < MT * NO; i += 256) {
    const int r = i / NO, c = i - r * NO;
    if (r0 + r < n) y[(r0 + r) * NO + c] = L.dy[r][c];
  }
}

// Count of set mask entries of the batch (a deterministic single-workgroup sum).
__global__ __launch_bounds__(256) void k_mask_count(const float* __restrict__ mask,
                                                    const int32_t* __restrict__ idx, int64_t n,
                                                    float* __restrict__ out) {
  __shared__ float red[256];
  float a = 0.0f;
  for (int64_t i = threadIdx.x; i < n * NO; i += 256) {
    const int64_t r = i / NO;
    a += mask[(idx ? (int64_t)idx[r] : r) * NO + (i - r * NO)];
  }
  red[threadIdx.x] = a;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

// Forward and backward of one tile of MT samples; gradient partials of the
// tile (and its share of the loss) go to gpart[tile][NPARAM + 1].
__global__ __launch_bounds__(256) void k_mlp_grad(const float* __restrict__ prm,
                                                  const float* __restrict__ x,
                                                  const float* __restrict__ t,
                                                  const float* __restrict__ mask,
                                                  const int32_t* __restrict__ idx, int64_t n,
                                                  const float* __restrict__ cnt_p,
                                                  float* __restrict__ gpart) {
  __shared__ MlpLds L;
  __shared__ float yv[MT][NO];
  __shared__ float d1[MT][NH];
  __shared__ float lred[256];
  const int64_t r0 = (int64_t)blockIdx.x * MT;
  mlp_load(L, prm, x, idx, n, r0);
  mlp_forward(L, yv);
  const float cnt = fmaxf(cnt_p[0], 1.0f);
  float lsum = 0.0f;
  for (int i = threadIdx.x; i < MT * NO; i += 256) {
    const int r = i / NO, c = i - r * NO;
    float d = 0.0f;
    if (r0 + r < n) {
      const int64_t row = idx ? (int64_t)idx[r0 + r] : r0 + r;
      const float m = mask[row * NO + c];
      const float res = m > 0.0f ? (yv[r][c] - t[row * NO + c]) * m : 0.0f;
      lsum += res * res;
      d = 2.0f * res / cnt;
    }
    L.dy[r][c] = d;
  }
  lred[threadIdx.x] = lsum;
  __syncthreads();
  float* g = gpart + (int64_t)blockIdx.x * (NPARAM + 1);
  // layer 3: gW3 = relu(z2)^T dy, gb3 = sum dy; dz2 = (dy W3^T) * [z2 > 0]
  for (int i = threadIdx.x; i < NH * NO; i += 256) {
    const int k = i / NO, c = i - k * NO;
    float a = 0.0f;
    for (int r = 0; r < MT; ++r) a = fmaf(fmaxf(L.z2[r][k], 0.0f), L.dy[r][c], a);
    g[OW3 + i] = a;
  }
  for (int c = threadIdx.x; c < NO; c += 256) {
    float a = 0.0f;
    for (int r = 0; r < MT; ++r) a += L.dy[r][c];
    g[OB3 + c] = a;
  }
  for (int i = threadIdx.x; i < MT * NH; i += 256) {
    const int r = i / NH, k = i - r * NH;
    float a = 0.0f;
    for (int c = 0; c < NO; ++c) a = fmaf(L.dy[r][c], L.w[OW3 + k * NO + c], a);
    d1[r][k] = L.z2[r][k] > 0.0f ? a : 0.0f;  // dz2
  }
  __syncthreads();
  // layer 2: gW2 = relu(z1)^T dz2, gb2; dz1 = (dz2 W2^T) * [z1 > 0] (into z2's slot)
  for (int i = threadIdx.x; i < NH * NH; i += 256) {
    const int k = i / NH, c = i - k * NH;
    float a = 0.0f;
    for (int r = 0; r < MT; ++r) a = fmaf(fmaxf(L.z1[r][k], 0.0f), d1[r][c], a);
    g[OW2 + i] = a;
  }
  for (int c = threadIdx.x; c < NH; c += 256) {
    float a = 0.0f;
    for (int r = 0; r < MT; ++r) a += d1[r][c];
    g[OB2 + c] = a;
  }
  for (int i = threadIdx.x; i < MT * NH; i += 256) {
    const int r = i / NH, k = i - r * NH;
    float a = 0.0f;
    for (int c = 0; c < NH; ++c) a = fmaf(d1[r][c], L.w[OW2 + k * NH + c], a);
    L.z2[r][k] = L.z1[r][k] > 0.0f ? a : 0.0f;  // dz1
  }
  __syncthreads();
  // layer 1: gW1 = x^T dz1, gb1
  for (int i = threadIdx.x; i < NI * NH; i += 256) {
    const int k = i / NH, c = i - k * NH;
    float a = 0.0f;
    for (int r = 0; r < MT; ++r) a = fmaf(L.x[r][k], L.z2[r][c], a);
    g[OW1 + i] = a;
  }
  for (int c = threadIdx.x; c < NH; c += 256) {
    float a = 0.0f;
    for (int r = 0; r < MT; ++r) a += L.z2[r][c];
    g[OB1 + c] = a;
  }
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) lred[threadIdx.x] += lred[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) g[NPARAM] = lred[0];
}

// Sum of the tile partials (tiles in order), Adam update of every parameter;
// loss = sum of squared masked residuals / count.
__global__ void k_mlp_adam(const float* __restrict__ gpart, int ntiles, float* __restrict__ prm,
                           float* __restrict__ m1, float* __restrict__ m2, float lr, float beta1,
                           float beta2, float eps, float c1, float c2,
                           const float* __restrict__ cnt_p, float* __restrict__ loss) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i > NPARAM) return;
  float g = 0.0f;
  for (int tl = 0; tl < ntiles; ++tl) g += gpart[(int64_t)tl * (NPARAM + 1) + i];
  if (i == NPARAM) {
    if (loss) loss[0] = g / fmaxf(cnt_p[0], 1.0f);
    return;
  }
  const float a = beta1 * m1[i] + (1.0f - beta1) * g;
  const float b = beta2 * m2[i] + (1.0f - beta2) * g * g;
  m1[i] = a;
  m2[i] = b;
  prm[i] -= lr * (a / c1) / (sqrtf(b / c2) + eps);
}

// s[b] = the smallest s in 1..8 with pred[b][s-1] <= log10(target), else 0.
__global__ void k_choose(const float* __restrict__ pred, int64_t n, double lt,
                         int32_t* __restrict__ s_out) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n) return;
  int s = 0;
  for (int k = NO; k >= 1; --k)
    if ((double)pred[b * NO + k - 1] <= lt) s = k;
  s_out[b] = s;
}

// err = |occ| max_{mu >= nu} |Kp[mu][nu] - Kref[mu][nu]| / kfro (lower triangles).
__global__ __launch_bounds__(256) void k_block_err(const double* __restrict__ Kp,
                                                   const double* __restrict__ Kref, int nao,
                                                   double scale, unsigned long long* __restrict__ err) {
  const int64_t nn = (int64_t)nao * nao;
  double m = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nn;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int mu = (int)(e / nao), nu = (int)(e - (int64_t)mu * nao);
    if (nu <= mu) m = fmax(m, fabs(Kp[e] - Kref[e]));
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) m = fmax(m, __shfl_xor(m, off));
  if ((threadIdx.x & 63) == 0)
    atomicMax(err, (unsigned long long)__double_as_longlong(m * scale));
}

__global__ void k_copy_f64(const double* __restrict__ a, int64_t n, double* __restrict__ b) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    b[i] = a[i];
}

inline unsigned gcap(int64_t n, int64_t c = 4096) {
  int64_t g = (n + 255) / 256;
  return (unsigned)(g < 1 ? 1 : (g > c ? c : g));
}

}  // namespace

int mlp_nparam() { return NPARAM; }

hipError_t launch_xstats_from(hipStream_t st, const unsigned long long* xmax, const double* xss,
                              int nb, int nao, int64_t nslot, double* out) {
  if (nb <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_xstats_from, dim3((unsigned)nb), dim3(64), 0, st, xmax, xss, nao, nslot,
                     out);
  return hipGetLastError();
}

hipError_t launch_seg_stats(hipStream_t st, const double* A, const double* A2, int64_t n,
                            int64_t seglen, int64_t rowlen, int64_t last_valid, double* partial,
                            int nsplit, double* out) {
  const int64_t nseg = (n + seglen - 1) / seglen;
  hipLaunchKernelGGL(k_seg_stats_partial, dim3((unsigned)nseg, (unsigned)nsplit), dim3(256), 0, st,
                     A, A2, n, seglen, rowlen, last_valid, nsplit, partial);
  hipLaunchKernelGGL(k_seg_stats_final, dim3((unsigned)((nseg + 255) / 256)), dim3(256), 0, st,
                     partial, nseg, nsplit, out);
  return hipGetLastError();
}

hipError_t launch_features(hipStream_t st, const double* bstats, const double* xstats,
                           const double* dstat, const double* cstat, const double* kstat,
                           const CtlScalars& sc, int nb, float* feat) {
  hipLaunchKernelGGL(k_features, dim3((unsigned)((nb + 63) / 64)), dim3(64), 0, st, bstats, xstats,
                     dstat, cstat, kstat, sc, nb, feat);
  return hipGetLastError();
}

hipError_t launch_mlp_forward(hipStream_t st, const float* prm, const float* x, int64_t n, float* y) {
  hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)((n + MT - 1) / MT)), dim3(256), 0, st, prm, x, n,
                     y);
  return hipGetLastError();
}

hipError_t launch_mlp_train(hipStream_t st, float* prm, float* m1, float* m2, int64_t step,
                            const float* x, const float* t, const float* mask, const int32_t* idx,
                            int64_t n, float lr, float* gpart, float* cnt, float* loss) {
  const int ntiles = (int)((n + MT - 1) / MT);
  hipLaunchKernelGGL(k_mask_count, dim3(1), dim3(256), 0, st, mask, idx, n, cnt);
  hipLaunchKernelGGL(k_mlp_grad, dim3((unsigned)ntiles), dim3(256), 0, st, prm, x, t, mask, idx, n,
                     cnt, gpart);
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = (float)(1.0 - pow(0.9, (double)step));
  const float c2 = (float)(1.0 - pow(0.999, (double)step));
  hipLaunchKernelGGL(k_mlp_adam, dim3((unsigned)((NPARAM + 1 + 255) / 256)), dim3(256), 0, st, gpart,
                     ntiles, prm, m1, m2, lr, b1, b2, 1e-8f, c1, c2, cnt, loss);
  return hipGetLastError();
}

hipError_t launch_choose(hipStream_t st, const float* pred, int64_t n, double target, int32_t* s) {
  hipLaunchKernelGGL(k_choose, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, pred, n,
                     log10(target), s);
  return hipGetLastError();
}

hipError_t launch_block_err(hipStream_t st, const double* Kp, const double* Kref, int nao,
                            double scale, double* err) {
  hipError_t e = launch_fill_u64(st, reinterpret_cast<unsigned long long*>(err), 1, 0ull);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_block_err, dim3(gcap((int64_t)nao * nao, 1024)), dim3(256), 0, st, Kp, Kref,
                     nao, scale, reinterpret_cast<unsigned long long*>(err));
  return hipGetLastError();
}

hipError_t launch_copy_f64(hipStream_t st, const double* a, int64_t n, double* b) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_f64, dim3(gcap(n)), dim3(256), 0, st, a, n, b);
  return hipGetLastError();
}

}  // namespace dfjk
