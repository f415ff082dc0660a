// Coulomb part (Eqs. 3-4), the exchange reduction across aux-block groups,
// the energies and the error bound.  These passes are HBM-bound streams over
// B (rho, J) or tiny reductions; all sums run in a fixed order (deterministic).
#include "dfjk_internal.h"

namespace dfjk {
namespace {

__device__ __forceinline__ double block_sum_256(double v, double* sh) {
  const int t = threadIdx.x;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
  if ((t & 63) == 0) sh[t >> 6] = v;
  __syncthreads();
  double r = 0.0;
  if (t == 0) r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  __syncthreads();
  return r;
}

// rho_P = sum_{mu,nu} B[P][mu][nu] D[mu][nu] (Eq. 3): one workgroup per P.
__global__ __launch_bounds__(256) void k_rho(const double* __restrict__ B, int64_t naux,
                                             int64_t nn, const double* __restrict__ D,
                                             double* __restrict__ rho) {
  __shared__ double sh[4];
  const int64_t P = blockIdx.x;
  const double* bp = B + P * nn;
  double acc0 = 0.0, acc1 = 0.0;
  const int t = threadIdx.x;
  if ((nn & 1) == 0) {
    const double2* b2 = reinterpret_cast<const double2*>(bp);
    const double2* d2 = reinterpret_cast<const double2*>(D);
    for (int64_t i = t; i < nn / 2; i += 256) {
      const double2 b = b2[i], d = d2[i];
      acc0 = fma(b.x, d.x, acc0);
      acc1 = fma(b.y, d.y, acc1);
    }
  } else {
    for (int64_t i = t; i < nn; i += 256) acc0 = fma(bp[i], D[i], acc0);
  }
  const double r = block_sum_256(acc0 + acc1, sh);
  if (t == 0) rho[P] = r;
}

// J partials (Eq. 4) over the lower triangle (J and every B_P are symmetric):
// Jp[split][mu][nu] = sum over P of the split (ascending) of rho_P B[P][mu][nu],
// nu <= mu.  Workgroup w takes rows w and nao - 1 - w, nao + 1 elements in
// all, so every workgroup streams the same number of bytes; thread t owns
// elements t, t + 256, ... of the two rows, concatenated.
// Packed B (packed != 0): B_P is its lower triangle by rows, element (mu, nu)
// at mu (mu + 1) / 2 + nu, so the two rows of a workgroup are contiguous.
template <int EPT>
__global__ __launch_bounds__(256) void k_j_tri(const double* __restrict__ B, int64_t naux, int nao,
                                               const double* __restrict__ rho, int jsplit,
                                               double* __restrict__ out, int mirror,
                                               const uint8_t* __restrict__ smask, int blk,
                                               int packed) {
  const int w = blockIdx.x;
  const int mu0 = w, mu1 = nao - 1 - w;
  const int n0 = mu0 + 1;
  const int ntot = mu1 > mu0 ? n0 + mu1 + 1 : n0;
  const int split = blockIdx.y;
  const int64_t p_lo = (int64_t)split * naux / jsplit, p_hi = (int64_t)(split + 1) * naux / jsplit;
  const int64_t nn = (int64_t)nao * nao;
  const int64_t pstride = packed ? (int64_t)nao * (nao + 1) / 2 : nn;  // per aux index
  for (int base = 0; base < ntot; base += 256 * EPT) {
    int64_t off[EPT], boff[EPT];
    bool ok[EPT], rd[EPT];
    const int nblk = (nao + blk - 1) / blk;
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
      const int idx = base + threadIdx.x + 256 * j;
      ok[j] = idx < ntot;
      const int mu = idx < n0 ? mu0 : mu1;
      const int nu = idx < n0 ? idx : idx - n0;
      off[j] = ok[j] ? (int64_t)mu * nao + nu : 0;
      boff[j] = ok[j] ? (packed ? (int64_t)mu * (mu + 1) / 2 + nu : off[j]) : 0;
      // a dropped shell block of the screened B is zero: its sum is 0
      rd[j] = ok[j] && (!smask || smask[(mu / blk) * nblk + nu / blk]);
    }
    double a[EPT];
#pragma unroll
    for (int j = 0; j < EPT; ++j) a[j] = 0.0;
    // four aux indices per step: 4 EPT independent loads in flight per lane
    int64_t P = p_lo;
    for (; P + 4 <= p_hi; P += 4) {
      double bv[4][EPT];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int j = 0; j < EPT; ++j) bv[u][j] = rd[j] ? B[(P + u) * pstride + boff[j]] : 0.0;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double r = rho[P + u];
#pragma unroll
        for (int j = 0; j < EPT; ++j)
          if (rd[j]) a[j] = fma(r, bv[u][j], a[j]);
      }
    }
    for (; P < p_hi; ++P) {
      const double r = rho[P];
      const double* bp = B + P * pstride;
#pragma unroll
      for (int j = 0; j < EPT; ++j)
        if (rd[j]) a[j] = fma(r, bp[boff[j]], a[j]);
    }
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
      if (!ok[j]) continue;
      out[split * nn + off[j]] = a[j];
      if (mirror) {
        const int64_t mu = off[j] / nao, nu = off[j] - mu * nao;
        out[nu * nao + mu] = a[j];
      }
    }
  }
}

// J[mu][nu] = J[nu][mu] = sum of the split partials (splits ascending), nu <= mu.
__global__ void k_sum_splits(const double* __restrict__ Jp, int jsplit, int nao,
                             double* __restrict__ J) {
  const int64_t nn = (int64_t)nao * nao;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nn;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int mu = (int)(e / nao), nu = (int)(e - (int64_t)mu * nao);
    if (nu > mu) continue;
    double v = 0.0;
    for (int s = 0; s < jsplit; ++s) v += Jp[s * nn + e];
    J[e] = v;
    J[(int64_t)nu * nao + mu] = v;
  }
}

// K[mu][nu] = K[nu][mu] = occ * sum_grp Kp[grp][mu][nu] (mu >= nu), groups ascending.
__global__ void k_k_reduce(const double* __restrict__ Kp, int groups, int nao, double occ,
                           double* __restrict__ K) {
  const int64_t nn = (int64_t)nao * nao;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nn;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int mu = (int)(e / nao), nu = (int)(e - (int64_t)mu * nao);
    if (mu < nu) continue;
    double v = 0.0;
    for (int g = 0; g < groups; ++g) v += Kp[g * nn + e];
    v *= occ;
    K[e] = v;
    K[(int64_t)nu * nao + mu] = v;
  }
}

// Fock matrix of the closed-shell SCF around the build (the paper's Sec. 4.3
// iterations): F = h + J - K / 2 elementwise ((h + J) first), and the partial
// sums of tr(D h) over fixed slices (256 workgroups, grid-stride), summed in
// order by k_sum_parts.
__global__ __launch_bounds__(256) void k_fock(const double* __restrict__ h,
                                              const double* __restrict__ J,
                                              const double* __restrict__ K,
                                              const double* __restrict__ D, int64_t nn,
                                              double* __restrict__ F, double* __restrict__ part) {
  __shared__ double sh[4];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < nn; i += (int64_t)gridDim.x * 256) {
    const double hv = h[i];
    F[i] = (hv + J[i]) - 0.5 * K[i];
    acc = fma(D[i], hv, acc);
  }
  const double r = block_sum_256(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = r;
}

__global__ void k_sum_parts(const double* __restrict__ part, int n, double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double v = 0.0;
  for (int i = 0; i < n; ++i) v += part[i];
  *out = v;
}

// Energies in two deterministic passes: 256 workgroups reduce fixed slices of
// rho^2 and D*K into scratch[2][256]; one workgroup then sums the partials in
// order.  energies[0] = 1/2 sum_P rho_P^2, energies[1] = -1/4 sum D K.
__global__ __launch_bounds__(256) void k_energy_partials(const double* __restrict__ rho,
                                                         int64_t naux,
                                                         const double* __restrict__ D,
                                                         const double* __restrict__ K, int64_t nn,
                                                         double* __restrict__ scratch) {
  __shared__ double sh[4];
  const int t = threadIdx.x, g = blockIdx.x;
  const int64_t stride = (int64_t)gridDim.x * 256;
  double a = 0.0, b = 0.0;
  for (int64_t i = (int64_t)g * 256 + t; i < naux; i += stride) a = fma(rho[i], rho[i], a);
  for (int64_t i = (int64_t)g * 256 + t; i < nn; i += stride) b = fma(D[i], K[i], b);
  const double sa = block_sum_256(a, sh);
  const double sb = block_sum_256(b, sh);
  if (t == 0) {
    scratch[g] = sa;
    scratch[256 + g] = sb;
  }
}

__global__ __launch_bounds__(256) void k_energy_final(const double* __restrict__ scratch,
                                                      double* __restrict__ energies) {
  __shared__ double sh[4];
  const int t = threadIdx.x;
  const double ej = block_sum_256(scratch[t], sh);
  const double ex = block_sum_256(scratch[256 + t], sh);
  if (t == 0) {
    energies[0] = 0.5 * ej;
    energies[1] = -0.25 * ex;
  }
}

// rho_P = sum_mu rowdot[P nao + mu], one wavefront per P, fixed lane order.
__global__ __launch_bounds__(256) void k_rho_reduce(const double* __restrict__ rowdot,
                                                    int64_t naux, int nao,
                                                    double* __restrict__ rho) {
  const int lane = threadIdx.x & 63;
  const int64_t P = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 6;
  if (P >= naux) return;
  const double* r = rowdot + P * nao;
  double a = 0.0;
  for (int mu = lane; mu < nao; mu += 64) a += r[mu];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) a += __shfl_xor(a, off);
  if (lane == 0) rho[P] = a;
}

// Per (block, mu): A = nao kappa1 Fsum sum_{P in b} 2^e_B, dmax = nao kappa1 Fmax
// max_{P in b} 2^e_B, pf = 2^F.  Fsum / Fmax over the orbital exponents f_i.
__global__ void k_bound_prep(const int32_t* __restrict__ b_exp, const int32_t* __restrict__ f_col,
                             int nocc, const int32_t* __restrict__ F, int fstride, int64_t naux,
                             int nao, int pblk, int nb, double kappa1,
                             const int32_t* __restrict__ sblk, double* __restrict__ scratch,
                             int extra) {
  double fsum = 0.0, fmx = 0.0;
  for (int i = 0; i < nocc; ++i) {
    const double v = ldexp(1.0, f_col[i]);
    fsum += v;
    fmx = fmax(fmx, v);
  }
  const int64_t n = (int64_t)nb * nao;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(idx / nao), mu = (int)(idx - (int64_t)b * nao);
    const int64_t p0 = (int64_t)b * pblk;
    const int64_t p1 = p0 + pblk < naux ? p0 + pblk : naux;
    const double k1 = sblk ? kappa_of(sblk[b], nao, extra) : kappa1;
    double se = 0.0, me = 0.0;
    // eight independent exponent loads in flight per step (the sum order is
    // unchanged: P ascending)
    int64_t P = p0;
    for (; P + 8 <= p1; P += 8) {
      int ex[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) ex[u] = b_exp[(P + u) * nao + mu];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const double v = ldexp(1.0, ex[u]);
        se += v;
        me = fmax(me, v);
      }
    }
    for (; P < p1; ++P) {
      const double v = ldexp(1.0, b_exp[P * nao + mu]);
      se += v;
      me = fmax(me, v);
    }
    scratch[3 * idx + 0] = nao * k1 * fsum * se;
    scratch[3 * idx + 1] = nao * k1 * fmx * me;
    scratch[3 * idx + 2] = ldexp(1.0, F[(int64_t)b * fstride + mu]);
  }
}

// bound(mu, nu) = |occ| [ sum_b (A_mu pf_nu + (pf_mu + dmax_mu) A_nu + kb pf_mu pf_nu kappa2_b)
//                 + (nb - 1) u (1 + u)^nb sum_b kb pf_mu pf_nu (1 + kappa2_b) ]
//                 (+ u |occ| kabs when occ is not a power of two); max over (mu, nu).
__global__ __launch_bounds__(256) void k_bound(const double* __restrict__ scratch, int nao, int nb,
                                               int64_t naux, int pblk, int nocc,
                                               double kappa2_full, double kappa2_last, double occ,
                                               int occ_pow2, const int32_t* __restrict__ sblk,
                                               double* __restrict__ err_bound, int extra) {
  // lane: one nu of the 256-wide column chunk blockIdx.x; the workgroup's
  // KB_ROWS rows mu (blockIdx.y) are the same for every lane, so each lane reads
  // its nu terms once per block and the mu terms are uniform loads
  constexpr int KB_ROWS = 8;
  const double u = 0x1p-53;
  const double accf = (nb - 1) * u * pow(1.0 + u, (double)nb);
  const int nu = blockIdx.x * 256 + threadIdx.x;
  const int mu0 = blockIdx.y * KB_ROWS;
  const bool live = nu < nao;
  const int nuc = live ? nu : 0;
  double sum[KB_ROWS], kabs[KB_ROWS];
#pragma unroll
  for (int m = 0; m < KB_ROWS; ++m) sum[m] = kabs[m] = 0.0;
  for (int b = 0; b < nb; ++b) {
    const double* sn = scratch + 3 * ((int64_t)b * nao + nuc);
    const double sn0 = sn[0], sn2 = sn[2];
    const int64_t p0 = (int64_t)b * pblk;
    const int64_t kb = ((p0 + pblk < naux ? p0 + pblk : naux) - p0) * nocc;
    const double k2 = sblk ? kappa_of(sblk[b], kb, extra) : (b == nb - 1 ? kappa2_last : kappa2_full);
#pragma unroll
    for (int m = 0; m < KB_ROWS; ++m) {
      const int mu = mu0 + m < nao ? mu0 + m : nao - 1;
      const double* sm = scratch + 3 * ((int64_t)b * nao + mu);
      const double pp = sm[2] * sn2;
      sum[m] += sm[0] * sn2 + (sm[2] + sm[1]) * sn0 + (double)kb * pp * k2;
      kabs[m] += (double)kb * pp * (1.0 + k2);
    }
  }
  double best = 0.0;
#pragma unroll
  for (int m = 0; m < KB_ROWS; ++m) {
    if (!live || mu0 + m >= nao) continue;
    double bound = fabs(occ) * (sum[m] + accf * kabs[m]);
    if (!occ_pow2) bound += u * fabs(occ) * kabs[m];
    best = fmax(best, bound);
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) best = fmax(best, __shfl_xor(best, off));
  if ((threadIdx.x & 63) == 0)
    atomicMax(reinterpret_cast<unsigned long long*>(err_bound),
              (unsigned long long)__double_as_longlong(best));
}

__global__ void k_zero_f64(double* p) { *p = 0.0; }

}  // namespace

hipError_t launch_rho(hipStream_t st, const double* B, int64_t naux, int nao, const double* D,
                      double* rho) {
  if (naux <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rho, dim3((unsigned)naux), dim3(256), 0, st, B, naux,
                     (int64_t)nao * nao, D, rho);
  return hipGetLastError();
}

hipError_t launch_j(hipStream_t st, const double* B, int64_t naux, int nao, const double* rho,
                    int jsplit, double* Jp, double* J, const uint8_t* smask, int blk, int packed) {
  const int64_t nn = (int64_t)nao * nao;
  const dim3 grid((unsigned)((nao + 1) / 2), (unsigned)jsplit);
  if (jsplit <= 1) {
    hipLaunchKernelGGL((k_j_tri<4>), grid, dim3(256), 0, st, B, naux, nao, rho, 1, J, 1, smask, blk,
                       packed);
    return hipGetLastError();
  }
  hipLaunchKernelGGL((k_j_tri<4>), grid, dim3(256), 0, st, B, naux, nao, rho, jsplit, Jp, 0, smask,
                     blk, packed);
  int64_t g = (nn + 255) / 256;
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(k_sum_splits, dim3((unsigned)g), dim3(256), 0, st, Jp, jsplit, nao, J);
  return hipGetLastError();
}

hipError_t launch_fock(hipStream_t st, const double* h, const double* J, const double* K,
                       const double* D, int64_t nao, double* F, double* scratch, double* e_one) {
  const int64_t nn = nao * nao;
  hipLaunchKernelGGL(k_fock, dim3(256), dim3(256), 0, st, h, J, K, D, nn, F, scratch);
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(64), 0, st, scratch, 256, e_one);
  return hipGetLastError();
}

hipError_t launch_k_reduce(hipStream_t st, const double* Kp, int groups, int nao, double occ,
                           double* K) {
  const int64_t nn = (int64_t)nao * nao;
  int64_t g = (nn + 255) / 256;
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(k_k_reduce, dim3((unsigned)g), dim3(256), 0, st, Kp, groups, nao, occ, K);
  return hipGetLastError();
}

hipError_t launch_energies(hipStream_t st, const double* rho, int64_t naux, const double* D,
                           const double* K, int nao, double* scratch, double* energies) {
  hipLaunchKernelGGL(k_energy_partials, dim3(256), dim3(256), 0, st, rho, naux, D, K,
                     (int64_t)nao * nao, scratch);
  hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(256), 0, st, scratch, energies);
  return hipGetLastError();
}

hipError_t launch_rho_reduce(hipStream_t st, const double* rowdot, int64_t naux, int nao,
                             double* rho) {
  if (naux <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rho_reduce, dim3((unsigned)((naux + 3) / 4)), dim3(256), 0, st, rowdot,
                     naux, nao, rho);
  return hipGetLastError();
}

hipError_t launch_bound(hipStream_t st, const int32_t* b_exp, const int32_t* f_col, int nocc,
                        const int32_t* F, int fstride, int64_t naux, int nao, int pblk, int nb,
                        double kappa1, double kappa2_full, double kappa2_last, double occ,
                        const int32_t* sblk, double* scratch, double* err_bound, int extra) {
  const int64_t n = (int64_t)nb * nao;
  int64_t g = (n + 255) / 256;
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(k_bound_prep, dim3((unsigned)g), dim3(256), 0, st, b_exp, f_col, nocc, F,
                     fstride, naux, nao, pblk, nb, kappa1, sblk, scratch, extra);
  hipLaunchKernelGGL(k_zero_f64, dim3(1), dim3(1), 0, st, err_bound);
  int occ_pow2 = 0;
  {
    int ex = 0;
    const double m = frexp(occ, &ex);
    occ_pow2 = (m == 0.5 || m == -0.5) ? 1 : 0;
  }
  // 256 columns nu by 8 rows mu per workgroup (the row count is k_bound's)
  const dim3 g2((unsigned)((nao + 255) / 256), (unsigned)((nao + 7) / 8));
  hipLaunchKernelGGL(k_bound, g2, dim3(256), 0, st, scratch, nao, nb, naux, pblk,
                     nocc, kappa2_full, kappa2_last, occ, occ_pow2, sblk, err_bound, extra);
  return hipGetLastError();
}

}  // namespace dfjk
