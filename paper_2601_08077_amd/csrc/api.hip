// C ABI of libdfjk: argument checks, workspace carving and the launch sequence
// of the density-fitting J/K build (Sec. 2.1 Eqs. 3-6, Sec. 3.2-3.3).
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/dfjk.h"
#include "dfjk_internal.h"

struct df_ctx {
  hipStream_t stream = nullptr;
  int slices = 0;
  int pblk = 64;
  int k_groups_req = 0;
  int k_groups_used = 0;
  // per-block statistics of X recorded by the last build's slicing of X
  // (valid for that shape and workspace only)
  bool xst_ok = false;
  int64_t xst_naux = 0, xst_nao = 0, xst_nocc = 0;
  int xst_pblk = 0;
  const char* xst_ws = nullptr;
  int x_ksub_req = 0;  // X chunk depth asked for (0 = autotuned or default)
  int extra = 0;       // anti-diagonals of digit pairs kept beyond a + b = s + 1
  int ncu = 256;  // compute units of the context's device
  int dev = -1;   // device current at df_create
  char* ws = nullptr;
  size_t ws_bytes = 0;
  int* status = nullptr;  // device word owned by the context
  std::string err;
  // stage timing: (DF_NSTAGES + 1) events per timed call
  std::vector<hipEvent_t> ev;
  int ev_cap = 0;
  int ev_used = 0;
  // per-aux-block slice counts (empty = the context precision for all blocks)
  std::vector<int32_t> blk_s;
  int32_t* blk_dev = nullptr;
  size_t blk_cap = 0;
  // small device scratch of the controller entry points (statistics partials,
  // perceptron gradient partials), allocated with the context
  char* aux = nullptr;
  // screening of B (caller-owned device arrays; null = dense)
  const uint8_t* scr_mask = nullptr;
  const unsigned long long* scr_chunks = nullptr;
  int scr_blk = 8;
  int64_t scr_nao = 0;
  // autotuned launch shapes per (naux, nao, nocc, slices, pblk): K groups, X chunk depth
  std::map<std::tuple<int64_t, int64_t, int64_t, int, int>, std::pair<int, int>> tuned;
  // worker streams of the batched build (created on first use, default
  // priority), their join events and the fork event
  std::vector<hipStream_t> workers;
  std::vector<hipEvent_t> joins;
  hipEvent_t fork = nullptr;
};

constexpr size_t kAuxBytes = (size_t)8 << 20;

// Workspace of df_build_jk_noalloc: one static array per device, held from
// the load of the library until the process ends.  Host code never passes the
// array's name to a kernel (on the host it is only a stand-in for the
// symbol); it uses the device address that df_create looks up once per
// device with that device current.
constexpr size_t kStaticWsBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) char scratch[kStaticWsBytes];
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

namespace {

using namespace dfjk;

int fail(df_ctx* c, int code, const char* msg) {
  if (c) c->err = msg;
  return code;
}

int hip_fail(df_ctx* c, hipError_t e, const char* where) {
  if (c) {
    c->err = std::string(where) + ": " + hipGetErrorString(e);
  }
  return DF_EHIP;
}

inline int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

// Every launcher reports hipGetLastError() after its launches, so an error
// left pending by some earlier runtime call of the host program (not of this
// library) is cleared on entry instead of being reported as ours.
inline void clear_stale_error() { (void)hipGetLastError(); }

// Shape-derived sizes shared by the workspace query and the build.
struct Plan {
  int64_t naux, nao, nocc;
  int pblk, nb, nao_pad, kbp, ncp, kp, groups, jsplit;
  int naux_pad, jdsplit;
  int packed;  // B stored as DF_PACKED (set by common_checks)
  size_t off_bexp, off_fcol, off_dC, off_X, off_xmax, off_F, off_Xd, off_rho, off_rowdot,
      off_Jp, off_Kp, off_bsc, off_esc, off_dD, off_gexp, off_h, off_wd, off_Sj, off_drho,
      off_Xs, off_Ks, off_xsmax, off_xss, total;
};

size_t carve(size_t& cur, size_t bytes) {
  const size_t o = cur;
  cur += (bytes + 255) / 256 * 256;
  return o;
}

// Default number of K partial groups: the count that minimises the K kernel's
// makespan in workgroup rounds, ceil(tiles g / slots) rounds of ceil(nb / g)
// aux blocks each (slots = workgroups resident on the device at once, taken
// at the largest slice count so that g, and with it the workspace size, does
// not depend on the slice count), the smallest such g.
static int default_k_groups(const df_ctx* c, int tiles, int nb) {
  const int64_t slots = (int64_t)c->ncu * k_int8_resident(kMaxSlices);
  int best = 1;
  int64_t best_cost = -1;
  for (int g = 1; g <= std::min(nb, 64); ++g) {
    const int64_t rounds = ((int64_t)tiles * g + slots - 1) / slots;
    const int64_t cost = rounds * ((nb + g - 1) / g);
    if (best_cost < 0 || cost < best_cost) {
      best_cost = cost;
      best = g;
    }
  }
  return best;
}

Plan make_plan(const df_ctx* c, int64_t naux, int64_t nao, int64_t nocc) {
  Plan p{};
  p.naux = naux;
  p.nao = nao;
  p.nocc = nocc;
  p.pblk = c->pblk;
  p.nb = (int)((naux + p.pblk - 1) / p.pblk);
  p.nao_pad = (int)round_up(nao, 64);
  p.kbp = (int)round_up((int64_t)p.pblk * nocc, 64);
  p.ncp = nocc <= 32 ? 32 : nocc <= 64 ? 64 : nocc <= 96 ? 96 : nocc <= 128 ? 128
                                                               : (int)round_up(nocc, 96);
  p.kp = (int)round_up(nao, 64);
  const int nt = p.nao_pad / 64;
  const int tiles = nt * (nt + 1) / 2;
  int g = c->k_groups_req;
  if (g <= 0) {
    const auto it = c->tuned.find(std::make_tuple(naux, nao, nocc, c->slices, c->pblk));
    g = it != c->tuned.end() ? it->second.first : default_k_groups(c, tiles, p.nb);
  }
  p.groups = std::max(1, std::min(g, p.nb));
  if (!c->blk_s.empty()) p.groups = p.nb;  // per-block precision: one partial per block
  const int64_t nn = nao * nao;
  {
    // J: (nao + 1) / 2 row-pair workgroups per aux split; aim at >= 4096 workgroups
    const int64_t pairs = (nao + 1) / 2;
    p.jsplit = (int)std::max<int64_t>(1, std::min<int64_t>(64, (4096 + pairs - 1) / pairs));
    p.jsplit = (int)std::min<int64_t>(p.jsplit, std::max<int64_t>(naux, 1));
  }
  size_t cur = 0;
  p.off_bexp = carve(cur, (size_t)naux * nao * 4);
  p.off_fcol = carve(cur, (size_t)std::max<int64_t>(nocc, 1) * 4);
  p.off_dC = carve(cur, (size_t)kMaxSlices * p.ncp * p.kp);
  p.off_X = carve(cur, (size_t)p.nb * p.pblk * nao * nocc * 8);  // blocked layout
  p.off_xmax = carve(cur, (size_t)p.nb * nao * 8);
  p.off_xss = carve(cur, (size_t)p.nb * (p.kbp / 64) * (p.nao_pad / 16) * 8);
  p.off_F = carve(cur, (size_t)p.nb * p.nao_pad * 4);
  p.off_Xd = carve(cur, (size_t)kMaxSlices * p.nb * p.nao_pad * p.kbp);
  p.off_rho = carve(cur, (size_t)naux * 8);
  p.off_rowdot = carve(cur, (size_t)naux * nao * 8);
  p.off_Jp = carve(cur, (size_t)(p.jsplit > 1 ? p.jsplit : 0) * nn * 8);
  p.off_Kp = carve(cur, (size_t)p.groups * nn * 8);
  p.off_bsc = carve(cur, (size_t)p.nb * nao * 3 * 8);
  p.off_esc = carve(cur, (size_t)512 * 8);
  // sliced mode: D digits, D row exponents, w exponents and digits, J's
  // integer sums, the per-P bound on rho
  p.naux_pad = (int)round_up(naux, 64);
  {
    const int64_t ngrp = (naux + 3) / 4;
    int64_t ns = std::max<int64_t>(1, (2048 + nao - 1) / nao);
    ns = std::min<int64_t>(ns, std::max<int64_t>(1, ngrp / 16));
    ns = std::max<int64_t>(ns, (naux * kMaxSlices + 65535) / 65536);
    p.jdsplit = (int)std::min<int64_t>(ns, 65535);
  }
  p.off_dD = carve(cur, (size_t)kMaxSlices * nao * p.kp);
  p.off_gexp = carve(cur, (size_t)nao * 4);
  p.off_h = carve(cur, (size_t)nao * 4);
  p.off_wd = carve(cur, (size_t)kMaxSlices * nao * p.naux_pad);
  p.off_Sj = carve(cur, (size_t)kMaxSlices * nn * 8);
  p.off_drho = carve(cur, (size_t)naux * 8 + 8);
  // FP64 check of sampled blocks: one block of X, one K partial, its row maxima
  p.off_Xs = carve(cur, (size_t)p.pblk * nao * nocc * 8);
  p.off_Ks = carve(cur, (size_t)nn * 8);
  p.off_xsmax = carve(cur, (size_t)nao * 8);
  p.total = cur;
  return p;
}

int check_shape(df_ctx* c, int layout, int64_t naux, int64_t nao, int64_t nocc) {
  if (!c) return DF_EINVAL;
  if (layout != DF_DENSE && layout != DF_PACKED)
    return fail(c, DF_EINVAL, "layout must be DF_DENSE or DF_PACKED");
  if (layout == DF_PACKED && nao > 16383)
    return fail(c, DF_EINVAL, "DF_PACKED supports nao <= 16383");
  if (naux < 1 || nao < 1 || nocc < 1) return fail(c, DF_EINVAL, "naux, nao and nocc must be >= 1");
  if (nao > 65536 || nocc > 65536 || naux > (int64_t)1 << 31)
    return fail(c, DF_EINVAL, "dimension too large");
  if (nocc > nao) return fail(c, DF_EINVAL, "nocc must not exceed nao");
  return DF_OK;
}

int check_guard(df_ctx* c, int s, int64_t nao, int64_t nocc) {
  if (s == 0) return DF_OK;
  const double lim = 2147483648.0;
  if ((double)s * (double)c->pblk * (double)nocc * 16384.0 >= lim)
    return fail(c, DF_EOVERFLOW_GUARD, "s * pblk * nocc * 2^14 >= 2^31: lower pblk");
  if ((double)s * (double)nao * 16384.0 >= lim)
    return fail(c, DF_EOVERFLOW_GUARD, "s * nao * 2^14 >= 2^31");
  return DF_OK;
}

template <class T>
T* at(df_ctx* c, size_t off) {
  return reinterpret_cast<T*>(c->ws + off);
}

// X chunk depth: the one set by df_set_x_ksub, else the autotuned one for
// this shape at the context precision, else 0 (the default).
int ksub_for(const df_ctx* c, int64_t naux, int64_t nao, int64_t nocc) {
  if (c->x_ksub_req) return c->x_ksub_req;
  const auto it = c->tuned.find(std::make_tuple(naux, nao, nocc, c->slices, c->pblk));
  return it != c->tuned.end() ? it->second.second : 0;
}

// Chunk and block masks of the screened B when they were set for this nao.
const unsigned long long* chunks_for(const df_ctx* c, int64_t nao) {
  return c->scr_chunks && c->scr_nao == nao ? c->scr_chunks : nullptr;
}
const uint8_t* mask_for(const df_ctx* c, int64_t nao) {
  return c->scr_mask && c->scr_nao == nao ? c->scr_mask : nullptr;
}

// Records the boundary event `idx` (0 = call start, i + 1 = end of stage i)
// of the current timed call, if timing is on and slots remain.
void mark(df_ctx* c, int idx) {
  if (c->ev_used >= c->ev_cap) return;
  (void)hipEventRecord(c->ev[(size_t)c->ev_used * (DF_NSTAGES + 1) + idx], c->stream);
}

#define DF_HIP(call, where)                       \
  do {                                            \
    hipError_t e_ = (call);                       \
    if (e_ != hipSuccess) return hip_fail(c, e_, where); \
  } while (0)

// squared-sum slots of X per aux block written by the slicing of X
int64_t xss_slots(const Plan& p) { return (int64_t)(p.kbp / 64) * (p.nao_pad / 16); }

void set_xstats(df_ctx* c, const Plan& p, bool ok) {
  c->xst_ok = ok;
  c->xst_naux = p.naux;
  c->xst_nao = p.nao;
  c->xst_nocc = p.nocc;
  c->xst_pblk = p.pblk;
  c->xst_ws = c->ws;
}

// X (and the per-(block, mu) max of |X|) at the context precision.
int run_x(df_ctx* c, const Plan& p, const double* B, const int32_t* b_exp, const double* C,
          double* X) {
  const int s = c->slices;
  unsigned long long* xmax = at<unsigned long long>(c, p.off_xmax);
  set_xstats(c, p, false);  // the workspace maxima now belong to the caller's X
  DF_HIP(launch_fill_u64(c->stream, xmax, (int64_t)p.nb * p.nao, 0ull), "fill xmax");
  if (s == 0) {
    DF_HIP(launch_x_fp64(c->stream, B, p.naux, (int)p.nao, C, (int)p.nocc, X, 0, xmax, p.pblk,
                         nullptr, nullptr, chunks_for(c, p.nao), p.packed),
           "x_fp64");
    return DF_OK;
  }
  int32_t* fcol = at<int32_t>(c, p.off_fcol);
  int8_t* dC = at<int8_t>(c, p.off_dC);
  DF_HIP(launch_col_exp(c->stream, C, p.nao, p.nocc, fcol, c->status), "col_exp");
  DF_HIP(launch_slice_c(c->stream, C, p.nao, p.nocc, s, fcol, p.ncp, p.kp, 0, dC), "slice_c");
  DF_HIP(launch_x_int8(c->stream, s, B, p.naux, (int)p.nao, b_exp, dC, p.ncp, p.kp, fcol,
                       (int)p.nocc, X, 0, xmax, p.pblk, nullptr, nullptr, chunks_for(c, p.nao),
                       ksub_for(c, p.naux, p.nao, p.nocc), nullptr, p.packed, c->extra),
         "x_int8");
  return DF_OK;
}

// Exponents and digits of X, the blocked K partials, their reduction (stages
// SLICE_X, K, K_REDUCE) at the context precision; X in the blocked layout.
int k_stages(df_ctx* c, const Plan& p, const double* X, double occ, double* K, int* fstride) {
  const int s = c->slices;
  hipStream_t st = c->stream;
  const int64_t naux = p.naux, nao = p.nao, nocc = p.nocc;
  unsigned long long* xmax = at<unsigned long long>(c, p.off_xmax);
  int32_t* F = at<int32_t>(c, p.off_F);
  double* Kp = at<double>(c, p.off_Kp);
  int8_t* Xd = at<int8_t>(c, p.off_Xd);
  if (s == 0) {
    DF_HIP(launch_xmax_to_exp(st, xmax, (int64_t)p.nb * nao, F), "xmax_to_exp");
    *fstride = (int)nao;
  } else {
    DF_HIP(launch_slice_x(st, s, X, naux, (int)nao, (int)nocc, p.pblk, p.nao_pad, p.kbp, xmax, F, Xd,
                          at<double>(c, p.off_xss)),
           "slice_x");
    *fstride = p.nao_pad;
  }
  // the per-block statistics of X come with the slicing (no FP64 path)
  set_xstats(c, p, s != 0);
  mark(c, 1 + DF_STAGE_SLICE_X);
  if (s == 0) {
    DF_HIP(launch_k_fp64(st, X, naux, (int)nao, (int)nocc, p.pblk, p.nb, p.groups, Kp), "k_fp64");
  } else {
    DF_HIP(launch_k_int8(st, s, Xd, F, p.nb, (int)nao, p.nao_pad, p.kbp, p.groups, Kp, nullptr,
                         c->extra),
           "k_int8");
  }
  mark(c, 1 + DF_STAGE_K);
  c->k_groups_used = p.groups;
  DF_HIP(launch_k_reduce(st, Kp, p.groups, (int)nao, occ, K), "k_reduce");
  mark(c, 1 + DF_STAGE_K_REDUCE);
  return DF_OK;
}

// Error bound of K into err_bound[0].  For s == 0 the FP64 X product is a
// length-nao dot product and each exchange partial is one accumulation chain
// of at most naux * nocc terms.
int k_bound_stage(df_ctx* c, const Plan& p, const int32_t* b_exp, const int32_t* fcol, int fstride,
                  double occ, double* err_bound) {
  const int s = c->slices;
  const int64_t naux = p.naux, nao = p.nao, nocc = p.nocc;
  const int64_t kb_full = (int64_t)p.pblk * nocc;
  const int64_t kb_last = (naux - (int64_t)(p.nb - 1) * p.pblk) * nocc;
  const double k1 = kappa_of(s, nao, c->extra);
  const double k2f = s ? kappa_of(s, kb_full, c->extra) : kappa_of(0, naux * nocc);
  const double k2l = s ? kappa_of(s, kb_last, c->extra) : kappa_of(0, naux * nocc);
  const int32_t* sblk = c->blk_s.empty() ? nullptr : c->blk_dev;
  DF_HIP(launch_bound(c->stream, b_exp, fcol, (int)nocc, at<int32_t>(c, p.off_F), fstride, naux,
                      (int)nao, p.pblk, p.nb, k1, k2f, k2l, occ, sblk, at<double>(c, p.off_bsc),
                      err_bound, c->extra),
         "bound");
  return DF_OK;
}

// Per-block precision: maximal runs [b0, b1) of consecutive aux blocks that
// share one slice count.
struct Run {
  int b0, b1, s;
};

std::vector<Run> block_runs(const df_ctx* c) {
  std::vector<Run> r;
  const int nb = (int)c->blk_s.size();
  for (int b = 0; b < nb;) {
    int e = b + 1;
    while (e < nb && c->blk_s[e] == c->blk_s[b]) ++e;
    r.push_back({b, e, c->blk_s[b]});
    b = e;
  }
  return r;
}

int effective_max_slices(const df_ctx* c) {
  if (c->blk_s.empty()) return c->slices;
  int m = 0;
  for (int v : c->blk_s) m = std::max(m, v);
  return m;
}

// X, its digits and the blocked K partials (one per block) with each run of
// blocks at its own slice count; the X, SLICE_X and K stage marks bracket
// the X pass and the interleaved slicing and K pass.
int xk_stages_blocks(df_ctx* c, const Plan& p, const double* B, const int32_t* b_exp,
                     const double* C, const double* D, double* rowdot, double occ, double* K,
                     int* fstride) {
  hipStream_t st = c->stream;
  const int64_t naux = p.naux, nao = p.nao, nocc = p.nocc, nn = nao * nao;
  double* X = at<double>(c, p.off_X);
  int32_t* fcol = at<int32_t>(c, p.off_fcol);
  int8_t* dC = at<int8_t>(c, p.off_dC);
  unsigned long long* xmax = at<unsigned long long>(c, p.off_xmax);
  int32_t* F = at<int32_t>(c, p.off_F);
  double* Kp = at<double>(c, p.off_Kp);
  int8_t* Xd = at<int8_t>(c, p.off_Xd);
  const std::vector<Run> runs = block_runs(c);
  for (const Run& r : runs) {
    const int64_t P0 = (int64_t)r.b0 * p.pblk;
    const int64_t P1 = std::min<int64_t>((int64_t)r.b1 * p.pblk, naux);
    const double* Bp = B + P0 * (p.packed ? nao * (nao + 1) / 2 : nn);
    double* Xr = X + P0 * nao * nocc;  // the blocked layout keeps each block contiguous
    if (r.s == 0) {
      DF_HIP(launch_x_fp64(st, Bp, P1 - P0, (int)nao, C, (int)nocc, Xr, 1, xmax + r.b0 * nao,
                           p.pblk, D, rowdot + P0 * nao, chunks_for(c, nao), p.packed),
             "x_fp64");
    } else {
      DF_HIP(launch_x_int8(st, r.s, Bp, P1 - P0, (int)nao, b_exp + P0 * nao, dC, p.ncp, p.kp, fcol,
                           (int)nocc, Xr, 1, xmax + r.b0 * nao, p.pblk, D, rowdot + P0 * nao,
                           chunks_for(c, nao), 0, nullptr, p.packed, c->extra),
             "x_int8");
    }
  }
  mark(c, 1 + DF_STAGE_X);
  mark(c, 1 + DF_STAGE_SLICE_X);
  for (const Run& r : runs) {
    const int64_t P0 = (int64_t)r.b0 * p.pblk;
    const int64_t P1 = std::min<int64_t>((int64_t)r.b1 * p.pblk, naux);
    const int nbr = r.b1 - r.b0;
    const double* Xr = X + P0 * nao * nocc;
    if (r.s == 0) {
      for (int b = r.b0; b < r.b1; ++b)
        DF_HIP(launch_xmax_to_exp(st, xmax + (int64_t)b * nao, nao, F + (int64_t)b * p.nao_pad),
               "xmax_to_exp");
      DF_HIP(launch_k_fp64(st, Xr, P1 - P0, (int)nao, (int)nocc, p.pblk, nbr, nbr,
                           Kp + (int64_t)r.b0 * nn),
             "k_fp64");
    } else {
      DF_HIP(launch_slice_x(st, r.s, Xr, P1 - P0, (int)nao, (int)nocc, p.pblk, p.nao_pad, p.kbp,
                            xmax + (int64_t)r.b0 * nao, F + (int64_t)r.b0 * p.nao_pad, Xd,
                            at<double>(c, p.off_xss) + (int64_t)r.b0 * xss_slots(p)),
             "slice_x");
      DF_HIP(launch_k_int8(st, r.s, Xd, F + (int64_t)r.b0 * p.nao_pad, nbr, (int)nao, p.nao_pad,
                           p.kbp, nbr, Kp + (int64_t)r.b0 * nn, nullptr, c->extra),
             "k_int8");
    }
  }
  mark(c, 1 + DF_STAGE_K);
  bool all_int8 = true;
  for (const Run& r : runs) all_int8 = all_int8 && r.s != 0;
  set_xstats(c, p, all_int8);
  c->k_groups_used = p.nb;
  DF_HIP(launch_k_reduce(st, Kp, p.nb, (int)nao, occ, K), "k_reduce");
  mark(c, 1 + DF_STAGE_K_REDUCE);
  *fstride = p.nao_pad;
  return DF_OK;
}

int common_checks(df_ctx* c, const double* B, int layout, int64_t naux, int64_t nao,
                  const double* C, int64_t nocc, Plan& p) {
  int rc = check_shape(c, layout, naux, nao, nocc);
  if (rc) return rc;
  if (!B || !C) return fail(c, DF_EINVAL, "null B or C");
  rc = check_guard(c, effective_max_slices(c), nao, nocc);
  if (rc) return rc;
  if (layout == DF_PACKED && chunks_for(c, nao))
    return fail(c, DF_EINVAL, "screening masks apply to DF_DENSE B only");
  p = make_plan(c, naux, nao, nocc);
  p.packed = layout == DF_PACKED;
  if (!c->ws || c->ws_bytes < p.total) return fail(c, DF_EWORKSPACE, "workspace too small");
  return DF_OK;
}

// Row exponents of B (dense or packed) into b_exp.
hipError_t launch_bexp(df_ctx* c, const double* B, int packed, int64_t naux, int64_t nao,
                       int32_t* b_exp) {
  if (packed) return launch_row_exp_packed(c->stream, B, naux, (int)nao, b_exp, c->status);
  return launch_row_exp(c->stream, B, naux * nao, nao, nao, b_exp, c->status);
}

}  // namespace

extern "C" {

int df_create(df_ctx** ctx, void* hip_stream) {
  clear_stale_error();
  if (!ctx) return DF_EINVAL;
  *ctx = nullptr;
  df_ctx* c = new df_ctx();
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) == hipSuccess) {
      c->dev = dev;
      if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0)
        c->ncu = n;
    }
    clear_stale_error();
  }
  if (c->dev >= 0 && c->dev < kMaxDevices) {
    // device address of this device's static workspace (once per device)
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[c->dev]) {
      void* ptr = nullptr;
      const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !ptr) {
        fprintf(stderr, "df_create: hipGetSymbolAddress(scratch): %s\n", hipGetErrorString(e));
        delete c;
        return DF_EHIP;
      }
      g_scratch_ptr[c->dev] = ptr;
    }
  }
  hipError_t e = hipMalloc(&c->status, 256);
  if (e != hipSuccess) {
    fprintf(stderr, "df_create: hipMalloc: %s\n", hipGetErrorString(e));
    delete c;
    return DF_EHIP;
  }
  e = hipMalloc(&c->aux, kAuxBytes);
  if (e != hipSuccess) {
    fprintf(stderr, "df_create: hipMalloc: %s\n", hipGetErrorString(e));
    (void)hipFree(c->status);
    delete c;
    return DF_EHIP;
  }
  e = launch_fill_i32(c->stream, c->status, 1, 0);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    fprintf(stderr, "df_create: status word: %s\n", hipGetErrorString(e));
    (void)hipFree(c->status);
    (void)hipFree(c->aux);
    delete c;
    return DF_EHIP;
  }
  *ctx = c;
  return DF_OK;
}

void df_destroy(df_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
  (void)hipFree(c->status);
  if (c->blk_dev) (void)hipFree(c->blk_dev);
  (void)hipFree(c->aux);
  for (hipStream_t w : c->workers) {
    (void)hipStreamSynchronize(w);
    (void)hipStreamDestroy(w);
  }
  for (hipEvent_t e : c->joins) (void)hipEventDestroy(e);
  if (c->fork) (void)hipEventDestroy(c->fork);
  delete c;
}

int df_set_precision(df_ctx* c, int slices) {
  if (!c) return DF_EINVAL;
  if (slices < 0 || slices > kMaxSlices) return fail(c, DF_EINVAL, "slices must be 0..8");
  c->slices = slices;
  return DF_OK;
}

int df_get_precision(const df_ctx* c) { return c ? c->slices : DF_EINVAL; }

int df_set_pblk(df_ctx* c, int pblk) {
  if (!c) return DF_EINVAL;
  if (pblk < 1 || pblk > 1024) return fail(c, DF_EINVAL, "pblk must be 1..1024");
  c->pblk = pblk;
  return DF_OK;
}

int df_set_k_groups(df_ctx* c, int groups) {
  if (!c) return DF_EINVAL;
  if (groups < 0 || groups > 4096) return fail(c, DF_EINVAL, "groups must be 0..4096");
  c->k_groups_req = groups;
  return DF_OK;
}

int df_set_block_precision(df_ctx* c, const int32_t* host_s, int64_t nblocks) {
  clear_stale_error();
  if (!c) return DF_EINVAL;
  if (!host_s) {
    c->blk_s.clear();
    return DF_OK;
  }
  if (nblocks < 1 || nblocks > (1 << 24)) return fail(c, DF_EINVAL, "nblocks must be 1..2^24");
  for (int64_t b = 0; b < nblocks; ++b)
    if (host_s[b] < 0 || host_s[b] > kMaxSlices) return fail(c, DF_EINVAL, "slice counts must be 0..8");
  if ((size_t)nblocks > c->blk_cap) {
    if (c->blk_dev) DF_HIP(hipFree(c->blk_dev), "hipFree");
    c->blk_dev = nullptr;
    c->blk_cap = 0;
    DF_HIP(hipMalloc(&c->blk_dev, (size_t)nblocks * sizeof(int32_t)), "hipMalloc");
    c->blk_cap = (size_t)nblocks;
  }
  // the stream may still read the previous counts
  DF_HIP(hipStreamSynchronize(c->stream), "sync");
  DF_HIP(hipMemcpy(c->blk_dev, host_s, (size_t)nblocks * sizeof(int32_t), hipMemcpyHostToDevice),
         "hipMemcpy");
  c->blk_s.assign(host_s, host_s + nblocks);
  return DF_OK;
}

int df_get_k_groups(const df_ctx* c) { return c ? c->k_groups_used : DF_EINVAL; }

int df_set_extra_pairs(df_ctx* c, int extra) {
  if (!c) return DF_EINVAL;
  if (extra < 0 || extra > 1) return fail(c, DF_EINVAL, "extra must be 0 or 1");
  c->extra = extra;
  return DF_OK;
}

int df_set_x_ksub(df_ctx* c, int ksub) {
  if (!c) return DF_EINVAL;
  if (ksub < 0 || ksub > 2) return fail(c, DF_EINVAL, "ksub must be 0, 1 or 2");
  c->x_ksub_req = ksub;
  return DF_OK;
}

int df_workspace_size(df_ctx* c, int64_t naux, int64_t nao, int64_t nocc, int layout,
                      size_t* bytes) {
  const int rc = check_shape(c, layout, naux, nao, nocc);
  if (rc) return rc;
  if (!bytes) return fail(c, DF_EINVAL, "null bytes");
  *bytes = make_plan(c, naux, nao, nocc).total;
  return DF_OK;
}

int df_set_workspace(df_ctx* c, void* dev_ptr, size_t bytes) {
  if (!c) return DF_EINVAL;
  if (dev_ptr && (reinterpret_cast<uintptr_t>(dev_ptr) & 255))
    return fail(c, DF_EINVAL, "workspace must be 256-byte aligned");
  c->ws = reinterpret_cast<char*>(dev_ptr);
  c->ws_bytes = dev_ptr ? bytes : 0;
  return DF_OK;
}

int df_b_exponents(df_ctx* c, const double* B, int layout, int64_t naux, int64_t nao,
                   int32_t* b_exp) {
  clear_stale_error();
  const int rc = check_shape(c, layout, naux, nao, 1);
  if (rc) return rc;
  if (!B || !b_exp) return fail(c, DF_EINVAL, "null pointer");
  DF_HIP(launch_bexp(c, B, layout == DF_PACKED, naux, nao, b_exp), "row_exp");
  return DF_OK;
}

int df_slice(df_ctx* c, const double* A, int64_t rows, int64_t cols, int64_t lda, int slices,
             int8_t* digits, int32_t* row_exp) {
  clear_stale_error();
  if (!c) return DF_EINVAL;
  if (!A || !digits || !row_exp) return fail(c, DF_EINVAL, "null pointer");
  if (rows < 0 || cols < 0 || lda < cols) return fail(c, DF_EINVAL, "bad rows/cols/lda");
  if (slices < 1 || slices > kMaxSlices) return fail(c, DF_EINVAL, "slices must be 1..8");
  if (rows == 0) return DF_OK;
  DF_HIP(launch_row_exp(c->stream, A, rows, cols, lda, row_exp, c->status), "row_exp");
  DF_HIP(launch_slice_rows(c->stream, A, rows, cols, lda, slices, row_exp, digits), "slice_rows");
  return DF_OK;
}

int df_build_x(df_ctx* c, const double* B, int layout, int64_t naux, int64_t nao,
               const int32_t* b_exp, const double* C, int64_t nocc, double* X) {
  clear_stale_error();
  Plan p;
  int rc = common_checks(c, B, layout, naux, nao, C, nocc, p);
  if (rc) return rc;
  if (!X) return fail(c, DF_EINVAL, "null X");
  if (c->slices > 0 && !b_exp) {
    int32_t* be = at<int32_t>(c, p.off_bexp);
    DF_HIP(launch_bexp(c, B, p.packed, naux, nao, be), "row_exp");
    b_exp = be;
  }
  return run_x(c, p, B, b_exp, C, X);
}

int df_build_jk(df_ctx* c, const double* B, int layout, int64_t naux, int64_t nao,
                const int32_t* b_exp, const double* C, int64_t nocc, double occ,
                const double* D, double* J, double* K, double* energies, double* err_bound) {
  clear_stale_error();
  Plan p;
  int rc = common_checks(c, B, layout, naux, nao, C, nocc, p);
  if (rc) return rc;
  if (!D || !J || !K || !energies || !err_bound) return fail(c, DF_EINVAL, "null output or D");
  if (!(occ == occ) || isinf(occ)) return fail(c, DF_EINVAL, "occ must be finite");
  const bool per_block = !c->blk_s.empty();
  if (per_block && (int64_t)c->blk_s.size() != p.nb)
    return fail(c, DF_EINVAL, "block precision set for another number of aux blocks");
  const int s = effective_max_slices(c);
  hipStream_t st = c->stream;
  mark(c, 0);
  if (!b_exp) {
    int32_t* be = at<int32_t>(c, p.off_bexp);
    DF_HIP(launch_bexp(c, B, p.packed, naux, nao, be), "row_exp");
    b_exp = be;
  }
  mark(c, 1 + DF_STAGE_BEXP);
  double* X = at<double>(c, p.off_X);
  int32_t* fcol = at<int32_t>(c, p.off_fcol);
  unsigned long long* xmax = at<unsigned long long>(c, p.off_xmax);
  DF_HIP(launch_fill_u64(st, xmax, (int64_t)p.nb * p.nao, 0ull), "fill xmax");
  DF_HIP(launch_col_exp(st, C, nao, nocc, fcol, c->status), "col_exp");
  int8_t* dC = at<int8_t>(c, p.off_dC);
  if (s > 0) DF_HIP(launch_slice_c(st, C, nao, nocc, s, fcol, p.ncp, p.kp, 0, dC), "slice_c");
  mark(c, 1 + DF_STAGE_PREP);
  // X in the blocked layout, with the B.D row dots of rho fused into the same pass over B
  double* rowdot = at<double>(c, p.off_rowdot);
  int fstride = 0;
  if (per_block) {
    rc = xk_stages_blocks(c, p, B, b_exp, C, D, rowdot, occ, K, &fstride);
    if (rc) return rc;
  } else if (s == 0) {
    DF_HIP(launch_x_fp64(st, B, naux, (int)nao, C, (int)nocc, X, 1, xmax, p.pblk, D, rowdot,
                         chunks_for(c, nao), p.packed),
           "x_fp64");
  } else {
    DF_HIP(launch_x_int8(st, s, B, naux, (int)nao, b_exp, dC, p.ncp, p.kp, fcol, (int)nocc, X, 1,
                         xmax, p.pblk, D, rowdot, chunks_for(c, nao), ksub_for(c, naux, nao, nocc),
                         nullptr, p.packed, c->extra),
           "x_int8");
  }
  if (!per_block) {
    mark(c, 1 + DF_STAGE_X);
    rc = k_stages(c, p, X, occ, K, &fstride);
    if (rc) return rc;
  }
  double* rho = at<double>(c, p.off_rho);
  DF_HIP(launch_rho_reduce(st, rowdot, naux, (int)nao, rho), "rho_reduce");
  mark(c, 1 + DF_STAGE_RHO);
  DF_HIP(launch_j(st, B, naux, (int)nao, rho, p.jsplit, at<double>(c, p.off_Jp), J,
                  mask_for(c, nao), c->scr_blk, p.packed),
         "j");
  mark(c, 1 + DF_STAGE_J);
  DF_HIP(launch_energies(st, rho, naux, D, K, (int)nao, at<double>(c, p.off_esc), energies),
         "energies");
  mark(c, 1 + DF_STAGE_ENERGIES);

  rc = k_bound_stage(c, p, b_exp, fcol, fstride, occ, err_bound);
  if (rc) return rc;
  mark(c, 1 + DF_STAGE_BOUND);
  if (c->ev_used < c->ev_cap) ++c->ev_used;
  return DF_OK;
}

int df_build_jk_noalloc(df_ctx* c, const double* B, int layout, int64_t naux, int64_t nao,
                        const int32_t* b_exp, const double* C, int64_t nocc, double occ,
                        const double* D, double* J, double* K, double* energies,
                        double* err_bound) {
  clear_stale_error();
  int rc = check_shape(c, layout, naux, nao, nocc);
  if (rc) return rc;
  void* ptr = nullptr;
  if (c->dev >= 0 && c->dev < kMaxDevices) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    ptr = g_scratch_ptr[c->dev];
  }
  if (!ptr) return fail(c, DF_EHIP, "no static workspace on the context's device");
  const size_t need = make_plan(c, naux, nao, nocc).total;
  if (need > kStaticWsBytes)
    return fail(c, DF_EWORKSPACE, "shape needs more than the 64 MiB static workspace");
  char* const saved_ws = c->ws;
  const size_t saved_bytes = c->ws_bytes;
  c->ws = reinterpret_cast<char*>(ptr);
  c->ws_bytes = kStaticWsBytes;
  rc = df_build_jk(c, B, layout, naux, nao, b_exp, C, nocc, occ, D, J, K, energies, err_bound);
  c->ws = saved_ws;
  c->ws_bytes = saved_bytes;
  return rc;
}

int df_prepare_b_size(int64_t naux, int64_t nao, int planes, size_t* bytes) {
  if (!bytes || naux < 1 || nao < 1 || nao > 65536 || planes < 1 || planes > kMaxSlices)
    return DF_EINVAL;
  *bytes = (size_t)planes * naux * nao * round_up(nao, 64);
  return DF_OK;
}

int df_prepare_b(df_ctx* c, const double* B, int layout, int64_t naux, int64_t nao, int planes,
                 int32_t* b_exp, int8_t* b_dig) {
  clear_stale_error();
  const int rc = check_shape(c, layout, naux, nao, 1);
  if (rc) return rc;
  if (!B || !b_exp || !b_dig) return fail(c, DF_EINVAL, "null pointer");
  if (planes < 1 || planes > kMaxSlices) return fail(c, DF_EINVAL, "planes must be 1..8");
  if (reinterpret_cast<uintptr_t>(b_dig) & 15) return fail(c, DF_EINVAL, "b_dig must be 16-byte aligned");
  DF_HIP(launch_bexp(c, B, layout == DF_PACKED, naux, nao, b_exp), "row_exp");
  DF_HIP(launch_slice_planes(c->stream, B, naux * nao, (int)nao, (int)round_up(nao, 64), b_exp,
                             planes, b_dig, layout == DF_PACKED),
         "slice_planes");
  return DF_OK;
}

int df_build_jk_sliced(df_ctx* c, const int8_t* b_dig, int planes, const int32_t* b_exp,
                       int64_t naux, int64_t nao, const double* C, int64_t nocc, double occ,
                       const double* D, double* J, double* K, double* energies,
                       double* err_bound) {
  clear_stale_error();
  int rc = check_shape(c, DF_DENSE, naux, nao, nocc);
  if (rc) return rc;
  const int s = c->slices;
  if (!c->blk_s.empty()) return fail(c, DF_EINVAL, "the sliced build uses one slice count: reset block precision");
  if (c->extra) return fail(c, DF_EINVAL, "the sliced build forms the plain digit pairs only: set extra pairs to 0");
  if (planes < 1 || planes > kMaxSlices) return fail(c, DF_EINVAL, "planes must be 1..8");
  if (s < 1 || s > planes) return fail(c, DF_EINVAL, "the sliced build needs 1 <= slices <= planes");
  if (!b_dig || !b_exp || !C || !D || !J || !K || !energies || !err_bound)
    return fail(c, DF_EINVAL, "null pointer");
  if (reinterpret_cast<uintptr_t>(b_dig) & 15) return fail(c, DF_EINVAL, "b_dig must be 16-byte aligned");
  if (!(occ == occ) || isinf(occ)) return fail(c, DF_EINVAL, "occ must be finite");
  rc = check_guard(c, s, nao, nocc);
  if (rc) return rc;
  const Plan p = make_plan(c, naux, nao, nocc);
  if (!c->ws || c->ws_bytes < p.total) return fail(c, DF_EWORKSPACE, "workspace too small");
  hipStream_t st = c->stream;
  const int ldk = p.kp;
  const int64_t bplane = naux * nao * ldk;
  mark(c, 0);
  mark(c, 1 + DF_STAGE_BEXP);
  double* X = at<double>(c, p.off_X);
  int32_t* fcol = at<int32_t>(c, p.off_fcol);
  int32_t* g = at<int32_t>(c, p.off_gexp);
  int8_t* dC = at<int8_t>(c, p.off_dC);
  int8_t* dD = at<int8_t>(c, p.off_dD);
  unsigned long long* xmax = at<unsigned long long>(c, p.off_xmax);
  DF_HIP(launch_fill_u64(st, xmax, (int64_t)p.nb * nao, 0ull), "fill xmax");
  DF_HIP(launch_col_exp(st, C, nao, nocc, fcol, c->status), "col_exp");
  DF_HIP(launch_slice_c(st, C, nao, nocc, s, fcol, p.ncp, p.kp, 1, dC), "slice_c");
  DF_HIP(launch_row_exp(st, D, nao, nao, nao, g, c->status), "row_exp D");
  DF_HIP(launch_slice_planes(st, D, nao, (int)nao, ldk, g, s, dD), "slice D");
  mark(c, 1 + DF_STAGE_PREP);
  double* rowdot = at<double>(c, p.off_rowdot);
  DF_HIP(launch_x_dig(st, s, b_dig, bplane, naux, (int)nao, ldk, b_exp, dC, p.ncp, fcol, (int)nocc,
                      X, xmax, p.pblk, dD, g, rowdot),
         "x_dig");
  mark(c, 1 + DF_STAGE_X);
  int fstride = 0;
  rc = k_stages(c, p, X, occ, K, &fstride);
  if (rc) return rc;
  double* rho = at<double>(c, p.off_rho);
  double* drho = at<double>(c, p.off_drho);
  const double u = ldexp(1.0, -53);
  const double kap_sum = (double)(nao - 1) * u * pow(1.0 + u, (double)nao);
  DF_HIP(launch_rho_seq(st, rowdot, b_exp, g, naux, (int)nao, kappa_of(s, nao), kap_sum, rho, drho),
         "rho_seq");
  mark(c, 1 + DF_STAGE_RHO);
  DF_HIP(launch_j_dig(st, s, b_dig, bplane, ldk, rho, drho, b_exp, naux, (int)nao, p.naux_pad,
                      p.jdsplit, kappa_of(s, naux), at<int32_t>(c, p.off_h), at<int8_t>(c, p.off_wd),
                      at<unsigned long long>(c, p.off_Sj),
                      reinterpret_cast<unsigned long long*>(err_bound + 1), J),
         "j_dig");
  mark(c, 1 + DF_STAGE_J);
  DF_HIP(launch_energies(st, rho, naux, D, K, (int)nao, at<double>(c, p.off_esc), energies),
         "energies");
  mark(c, 1 + DF_STAGE_ENERGIES);
  rc = k_bound_stage(c, p, b_exp, fcol, fstride, occ, err_bound);
  if (rc) return rc;
  mark(c, 1 + DF_STAGE_BOUND);
  if (c->ev_used < c->ev_cap) ++c->ev_used;
  return DF_OK;
}

// ---------------------------------------------------------------- controller
int seg_stats(df_ctx* c, const double* A, const double* A2, int64_t n, int64_t seglen,
              int64_t rowlen, int64_t last_valid, double* out) {
  const int64_t nseg = (n + seglen - 1) / seglen;
  const int64_t cap = (int64_t)(kAuxBytes / 16);
  if (nseg > cap) return fail(c, DF_EINVAL, "too many segments");
  const int nsplit = (int)std::max<int64_t>(1, std::min<int64_t>(64, cap / nseg));
  DF_HIP(launch_seg_stats(c->stream, A, A2, n, seglen, rowlen, last_valid,
                          reinterpret_cast<double*>(c->aux), nsplit, out),
         "seg_stats");
  return DF_OK;
}

int df_block_stats(df_ctx* c, const double* A, const double* A2, int64_t n, int64_t seglen,
                   double* out) {
  clear_stale_error();
  if (!c) return DF_EINVAL;
  if (!A || !out || n < 1 || seglen < 1) return fail(c, DF_EINVAL, "bad arguments");
  return seg_stats(c, A, A2, n, seglen, seglen, seglen, out);
}

int df_x_block_stats(df_ctx* c, int64_t naux, int64_t nao, int64_t nocc, double* out) {
  clear_stale_error();
  const int rc = check_shape(c, DF_DENSE, naux, nao, nocc);
  if (rc) return rc;
  if (!out) return fail(c, DF_EINVAL, "null out");
  const Plan p = make_plan(c, naux, nao, nocc);
  if (!c->ws || c->ws_bytes < p.total) return fail(c, DF_EWORKSPACE, "workspace too small");
  if (c->xst_ok && c->xst_ws == c->ws && c->xst_naux == naux && c->xst_nao == nao &&
      c->xst_nocc == nocc && c->xst_pblk == p.pblk) {
    // recorded by the build: the maxima of its X pass, the squares summed by its slicing
    DF_HIP(launch_xstats_from(c->stream, at<unsigned long long>(c, p.off_xmax),
                              at<double>(c, p.off_xss), p.nb, (int)nao, xss_slots(p), out),
           "xstats_from");
    return DF_OK;
  }
  // blocked X: block b holds rows mu of pblk * nocc entries; the last block
  // uses only its first (naux - (nb - 1) pblk) * nocc entries of each row
  const int64_t rowlen = (int64_t)p.pblk * nocc;
  const int64_t last_valid = (naux - (int64_t)(p.nb - 1) * p.pblk) * nocc;
  return seg_stats(c, at<double>(c, p.off_X), nullptr, (int64_t)p.nb * rowlen * nao, rowlen * nao,
                   rowlen, last_valid, out);
}

int df_controller_features(df_ctx* c, const double* bstats, const double* xstats,
                           const double* dstat, const double* cstat, const double* kstat,
                           const double* host_scalars, int64_t nblocks, float* feat) {
  clear_stale_error();
  if (!c) return DF_EINVAL;
  if (!bstats || !xstats || !dstat || !cstat || !kstat || !host_scalars || !feat || nblocks < 1)
    return fail(c, DF_EINVAL, "bad arguments");
  CtlScalars sc;
  sc.iteration = host_scalars[0];
  sc.n_iter = host_scalars[1];
  sc.de_rel = host_scalars[2];
  sc.target = host_scalars[3];
  sc.nao = host_scalars[4];
  sc.naux = host_scalars[5];
  sc.nocc = host_scalars[6];
  sc.plain_s = host_scalars[7];
  if (!(sc.n_iter > 0) || !(sc.nao >= 1) || !(sc.naux >= 1) || !(sc.nocc >= 1))
    return fail(c, DF_EINVAL, "n_iter, nao, naux, nocc must be positive");
  DF_HIP(launch_features(c->stream, bstats, xstats, dstat, cstat, kstat, sc, (int)nblocks, feat),
         "features");
  return DF_OK;
}

int df_mlp_nparams(void) { return mlp_nparam(); }

int df_mlp_forward(df_ctx* c, const float* params, const float* x, int64_t n, float* y) {
  clear_stale_error();
  if (!c) return DF_EINVAL;
  if (!params || !x || !y || n < 1 || n > ((int64_t)1 << 30)) return fail(c, DF_EINVAL, "bad arguments");
  DF_HIP(launch_mlp_forward(c->stream, params, x, n, y), "mlp_forward");
  return DF_OK;
}

int df_mlp_train_step(df_ctx* c, float* params, float* adam_m, float* adam_v, int64_t step,
                      const float* x, const float* t, const float* mask, const int32_t* idx,
                      int64_t n, float lr, float* loss) {
  clear_stale_error();
  if (!c) return DF_EINVAL;
  if (!params || !adam_m || !adam_v || !x || !t || !mask || step < 1 || n < 1)
    return fail(c, DF_EINVAL, "bad arguments");
  const int64_t ntiles = (n + 31) / 32;
  const size_t need = (size_t)ntiles * (mlp_nparam() + 1) * 4 + 256;
  if (need > kAuxBytes) return fail(c, DF_EINVAL, "batch too large (n <= 11000)");
  if (!(lr > 0.0f)) return fail(c, DF_EINVAL, "lr must be positive");
  float* cnt = reinterpret_cast<float*>(c->aux);
  float* gpart = reinterpret_cast<float*>(c->aux + 256);
  DF_HIP(launch_mlp_train(c->stream, params, adam_m, adam_v, step, x, t, mask, idx, n, lr, gpart, cnt,
                          loss),
         "mlp_train");
  return DF_OK;
}

int df_choose_slices(df_ctx* c, const float* pred, int64_t n, double target, int32_t* s_out) {
  clear_stale_error();
  if (!c) return DF_EINVAL;
  if (!pred || !s_out || n < 1) return fail(c, DF_EINVAL, "bad arguments");
  if (!(target > 0.0) || isinf(target)) return fail(c, DF_EINVAL, "target must be positive and finite");
  DF_HIP(launch_choose(c->stream, pred, n, target, s_out), "choose");
  return DF_OK;
}

int df_block_partials(df_ctx* c, int64_t naux, int64_t nao, int64_t nocc, double* out) {
  clear_stale_error();
  const int rc = check_shape(c, DF_DENSE, naux, nao, nocc);
  if (rc) return rc;
  if (!out) return fail(c, DF_EINVAL, "null out");
  if (c->blk_s.empty()) return fail(c, DF_EINVAL, "block partials exist only with block precision set");
  const Plan p = make_plan(c, naux, nao, nocc);
  if (!c->ws || c->ws_bytes < p.total) return fail(c, DF_EWORKSPACE, "workspace too small");
  DF_HIP(launch_copy_f64(c->stream, at<double>(c, p.off_Kp), (int64_t)p.nb * nao * nao, out), "copy");
  return DF_OK;
}

int df_block_errors(df_ctx* c, int64_t naux, int64_t nao, int64_t nocc, double occ,
                    const double* kref, double kfro, double* err) {
  clear_stale_error();
  const int rc = check_shape(c, DF_DENSE, naux, nao, nocc);
  if (rc) return rc;
  if (!kref || !err) return fail(c, DF_EINVAL, "null pointer");
  if (!(kfro > 0.0) || isinf(kfro)) return fail(c, DF_EINVAL, "kfro must be positive and finite");
  if (c->blk_s.empty()) return fail(c, DF_EINVAL, "block partials exist only with block precision set");
  const Plan p = make_plan(c, naux, nao, nocc);
  if (!c->ws || c->ws_bytes < p.total) return fail(c, DF_EWORKSPACE, "workspace too small");
  const int64_t nn = nao * nao;
  for (int b = 0; b < p.nb; ++b)
    DF_HIP(launch_block_err(c->stream, at<double>(c, p.off_Kp) + b * nn, kref + b * nn, (int)nao,
                            fabs(occ) / kfro, err + b),
           "block_err");
  return DF_OK;
}

int df_spot_check(df_ctx* c, const double* B, int layout, int64_t naux, int64_t nao,
                  const double* C, int64_t nocc, double occ, double kfro,
                  const int32_t* host_blocks, int nsample, double* err) {
  clear_stale_error();
  const int rc = check_shape(c, layout, naux, nao, nocc);
  if (rc) return rc;
  if (!B || !C || !host_blocks || !err || nsample < 1) return fail(c, DF_EINVAL, "bad arguments");
  if (!(kfro > 0.0) || isinf(kfro)) return fail(c, DF_EINVAL, "kfro must be positive and finite");
  if (c->blk_s.empty()) return fail(c, DF_EINVAL, "block partials exist only with block precision set");
  const Plan p = make_plan(c, naux, nao, nocc);
  if (!c->ws || c->ws_bytes < p.total) return fail(c, DF_EWORKSPACE, "workspace too small");
  for (int i = 0; i < nsample; ++i)
    if (host_blocks[i] < 0 || host_blocks[i] >= p.nb) return fail(c, DF_EINVAL, "block index out of range");
  hipStream_t st = c->stream;
  const int64_t nn = nao * nao;
  const int64_t bstride = layout == DF_PACKED ? nao * (nao + 1) / 2 : nn;  // per aux index
  double* Xs = at<double>(c, p.off_Xs);
  double* Ks = at<double>(c, p.off_Ks);
  unsigned long long* xm = at<unsigned long long>(c, p.off_xsmax);
  for (int i = 0; i < nsample; ++i) {
    const int b = host_blocks[i];
    const int64_t P0 = (int64_t)b * p.pblk;
    const int64_t P1 = std::min<int64_t>(P0 + p.pblk, naux);
    DF_HIP(launch_fill_u64(st, xm, nao, 0ull), "fill");
    DF_HIP(launch_x_fp64(st, B + P0 * bstride, P1 - P0, (int)nao, C, (int)nocc, Xs, 1, xm,
                         p.pblk, nullptr, nullptr, nullptr, layout == DF_PACKED),
           "x_fp64");
    DF_HIP(launch_k_fp64(st, Xs, P1 - P0, (int)nao, (int)nocc, p.pblk, 1, 1, Ks), "k_fp64");
    DF_HIP(launch_block_err(st, at<double>(c, p.off_Kp) + b * nn, Ks, (int)nao, fabs(occ) / kfro,
                            err + i),
           "block_err");
  }
  return DF_OK;
}

int df_screen(df_ctx* c, double* B, int64_t naux, int64_t nao, int blk, double tau, uint8_t* mask,
              uint64_t* chunks, double* norms) {
  clear_stale_error();
  const int rc = check_shape(c, DF_DENSE, naux, nao, 1);
  if (rc) return rc;
  if (!B || !mask || !chunks) return fail(c, DF_EINVAL, "null pointer");
  if (blk < 1 || blk > 64 || 64 % blk) return fail(c, DF_EINVAL, "blk must divide 64");
  if (nao > 4096) return fail(c, DF_EINVAL, "screening supports nao <= 4096");
  if (!(tau >= 0.0) || isinf(tau)) return fail(c, DF_EINVAL, "tau must be finite and >= 0");
  const int64_t nblk = (nao + blk - 1) / blk;
  const size_t per_split = (size_t)nblk * nao * 8;
  double* part;
  int nsplit;
  if (per_split <= kAuxBytes) {
    part = reinterpret_cast<double*>(c->aux);
    nsplit = (int)std::min<int64_t>({(int64_t)(kAuxBytes / per_split), 64,
                                     std::max<int64_t>(1, (1024 + nblk - 1) / nblk), naux});
  } else {
    if (!c->ws || c->ws_bytes < per_split)
      return fail(c, DF_EWORKSPACE, "screening needs a workspace of nblk * nao * 8 bytes");
    part = reinterpret_cast<double*>(c->ws);
    nsplit = 1;
  }
  DF_HIP(launch_screen(c->stream, B, naux, (int)nao, blk, tau, nsplit, part, norms, mask,
                       reinterpret_cast<unsigned long long*>(chunks)),
         "screen");
  return DF_OK;
}

int df_set_screening(df_ctx* c, const uint8_t* mask, const uint64_t* chunks, int blk, int64_t nao) {
  if (!c) return DF_EINVAL;
  if (!mask || !chunks) {
    c->scr_mask = nullptr;
    c->scr_chunks = nullptr;
    c->scr_nao = 0;
    return DF_OK;
  }
  if (blk < 1 || blk > 64 || 64 % blk) return fail(c, DF_EINVAL, "blk must divide 64");
  if (nao < 1 || nao > 4096) return fail(c, DF_EINVAL, "screening supports nao <= 4096");
  c->scr_mask = mask;
  c->scr_chunks = reinterpret_cast<const unsigned long long*>(chunks);
  c->scr_blk = blk;
  c->scr_nao = nao;
  return DF_OK;
}

// ------------------------------------------------------------- autotuning
int df_autotune(df_ctx* c, const double* B, const int32_t* b_exp, int64_t naux, int64_t nao,
                const double* C, int64_t nocc, double occ, const double* D, double* J, double* K,
                double* energies, double* err_bound, int reps, int* best_groups, int* best_ksub,
                double* best_ms) {
  clear_stale_error();
  int rc = check_shape(c, DF_DENSE, naux, nao, nocc);
  if (rc) return rc;
  if (reps < 1 || reps > 100) return fail(c, DF_EINVAL, "reps must be 1..100");
  if (!c->blk_s.empty()) return fail(c, DF_EINVAL, "autotuning needs uniform precision");
  const auto key = std::make_tuple(naux, nao, nocc, c->slices, c->pblk);
  c->tuned.erase(key);
  const int saved_req = c->k_groups_req, saved_ksub = c->x_ksub_req;
  c->k_groups_req = 0;
  c->x_ksub_req = 0;
  const Plan base = make_plan(c, naux, nao, nocc);
  std::vector<int> groups = {base.groups};
  for (int g = 1; g <= std::min(base.nb, 64); g *= 2)
    if (g != base.groups) groups.push_back(g);
  std::vector<int> ksubs = {1};
  if (c->slices >= 1 && c->slices <= 5 && nao % 128 == 0) ksubs.push_back(2);
  hipEvent_t e0, e1;
  DF_HIP(hipEventCreate(&e0), "hipEventCreate");
  DF_HIP(hipEventCreate(&e1), "hipEventCreate");
  const int saved_cap = c->ev_cap;
  c->ev_cap = 0;  // no stage marks while tuning
  double best = 1e300;
  std::pair<int, int> pick = {base.groups, 0};
  rc = DF_OK;
  for (int g : groups) {
    for (int ks : ksubs) {
      c->tuned[key] = {g, ks};
      const Plan p = make_plan(c, naux, nao, nocc);
      if (!c->ws || c->ws_bytes < p.total) continue;  // needs more workspace than given
      rc = df_build_jk(c, B, DF_DENSE, naux, nao, b_exp, C, nocc, occ, D, J, K, energies, err_bound);
      if (rc) break;
      hipError_t e = hipEventRecord(e0, c->stream);
      for (int r = 0; r < reps && e == hipSuccess && rc == DF_OK; ++r)
        rc = df_build_jk(c, B, DF_DENSE, naux, nao, b_exp, C, nocc, occ, D, J, K, energies, err_bound);
      if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e != hipSuccess) rc = hip_fail(c, e, "autotune timing");
      if (rc) break;
      if (ms / reps < best) {
        best = ms / reps;
        pick = {g, ks};
      }
    }
    if (rc) break;
  }
  c->ev_cap = saved_cap;
  c->k_groups_req = saved_req;
  c->x_ksub_req = saved_ksub;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) {
    c->tuned.erase(key);
    return rc;
  }
  if (best >= 1e300) return fail(c, DF_EWORKSPACE, "workspace too small for every candidate");
  c->tuned[key] = pick;
  if (best_groups) *best_groups = pick.first;
  if (best_ksub) *best_ksub = pick.second;
  if (best_ms) *best_ms = best;
  return DF_OK;
}

// ------------------------------------------------------------- batched build
namespace {

double instance_cost(const df_problem& q) {
  const double nn = (double)q.nao * q.nao;
  const double pairs = q.slices ? q.slices * (q.slices + 1) / 2.0 : 8.0;
  return nn * q.naux * (3.0 * q.nocc * pairs / 8.0 + 16.0);
}

// LPT: instances by cost, largest first, each onto the least-loaded stream.
std::vector<std::vector<int>> assign(int n, const df_problem* q, int streams) {
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return instance_cost(q[a]) > instance_cost(q[b]); });
  std::vector<std::vector<int>> out(streams);
  std::vector<double> load(streams, 0.0);
  for (int i : order) {
    const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    out[k].push_back(i);
    load[k] += instance_cost(q[i]);
  }
  return out;
}

int batched_plan(df_ctx* c, int n, const df_problem* probs, int streams,
                 std::vector<std::vector<int>>& groups, std::vector<size_t>& off, size_t& total) {
  if (!c) return DF_EINVAL;
  if (n < 1 || !probs) return fail(c, DF_EINVAL, "n >= 1 problems required");
  if (streams < 1 || streams > 4) return fail(c, DF_EINVAL, "streams must be 1..4");
  if (!c->blk_s.empty()) return fail(c, DF_EINVAL, "the batched build uses per-instance precision");
  const int saved = c->slices;
  for (int i = 0; i < n; ++i) {
    const df_problem& q = probs[i];
    int rc = check_shape(c, DF_DENSE, q.naux, q.nao, q.nocc);
    if (rc) return rc;
    if (q.slices < 0 || q.slices > kMaxSlices) return fail(c, DF_EINVAL, "slices must be 0..8");
    if (!q.B || !q.C || !q.D || !q.J || !q.K || !q.energies || !q.err_bound)
      return fail(c, DF_EINVAL, "null pointer in a problem");
    rc = check_guard(c, q.slices, q.nao, q.nocc);
    if (rc) return rc;
  }
  groups = assign(n, probs, streams);
  off.assign(streams, 0);
  total = 0;
  for (int k = 0; k < streams; ++k) {
    size_t need = 0;
    for (int i : groups[k]) {
      c->slices = probs[i].slices;
      need = std::max(need, make_plan(c, probs[i].naux, probs[i].nao, probs[i].nocc).total);
    }
    off[k] = total;
    total += (need + 255) / 256 * 256;
  }
  c->slices = saved;
  return DF_OK;
}

}  // namespace

int df_batched_workspace_size(df_ctx* c, int n, const df_problem* probs, int streams,
                              size_t* bytes) {
  std::vector<std::vector<int>> groups;
  std::vector<size_t> off;
  size_t total = 0;
  const int rc = batched_plan(c, n, probs, streams, groups, off, total);
  if (rc) return rc;
  if (!bytes) return fail(c, DF_EINVAL, "null bytes");
  *bytes = total;
  return DF_OK;
}

int df_build_jk_batched(df_ctx* c, int n, const df_problem* probs, int streams) {
  clear_stale_error();
  std::vector<std::vector<int>> groups;
  std::vector<size_t> off;
  size_t total = 0;
  int rc = batched_plan(c, n, probs, streams, groups, off, total);
  if (rc) return rc;
  if (!c->ws || c->ws_bytes < total) return fail(c, DF_EWORKSPACE, "workspace too small");
  // worker streams (default priority) and their fork / join events
  if (streams > 1 && !c->fork)
    DF_HIP(hipEventCreateWithFlags(&c->fork, hipEventDisableTiming), "hipEventCreate");
  while (streams > 1 && (int)c->workers.size() < streams) {
    hipStream_t w;
    DF_HIP(hipStreamCreateWithFlags(&w, hipStreamNonBlocking), "hipStreamCreate");
    c->workers.push_back(w);
    hipEvent_t e;
    DF_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreate");
    c->joins.push_back(e);
  }
  hipStream_t home = c->stream;
  char* ws = c->ws;
  const size_t ws_bytes = c->ws_bytes;
  const int saved_s = c->slices, saved_cap = c->ev_cap;
  const uint8_t* saved_mask = c->scr_mask;
  const unsigned long long* saved_chunks = c->scr_chunks;
  const int saved_blk = c->scr_blk;
  const int64_t saved_nao = c->scr_nao;
  c->ev_cap = 0;
  if (streams > 1) {
    hipError_t e = hipEventRecord(c->fork, home);
    for (int k = 0; k < streams && e == hipSuccess; ++k) e = hipStreamWaitEvent(c->workers[k], c->fork, 0);
    if (e != hipSuccess) {
      c->ev_cap = saved_cap;
      return hip_fail(c, e, "fork");
    }
  }
  for (int k = 0; k < streams && rc == DF_OK; ++k) {
    c->stream = streams > 1 ? c->workers[k] : home;
    c->ws = ws + off[k];
    c->ws_bytes = (k + 1 < streams ? off[k + 1] : total) - off[k];
    for (int i : groups[k]) {
      const df_problem& q = probs[i];
      c->slices = q.slices;
      c->scr_mask = q.screen_mask;
      c->scr_chunks = reinterpret_cast<const unsigned long long*>(q.screen_chunks);
      c->scr_blk = q.screen_blk > 0 ? q.screen_blk : 8;
      c->scr_nao = q.screen_mask ? q.nao : 0;
      rc = df_build_jk(c, q.B, DF_DENSE, q.naux, q.nao, q.b_exp, q.C, q.nocc, q.occ, q.D, q.J, q.K,
                       q.energies, q.err_bound);
      if (rc) break;
    }
  }
  if (streams > 1) {
    for (int k = 0; k < streams; ++k) {
      const hipError_t e1 = hipEventRecord(c->joins[k], c->workers[k]);
      const hipError_t e2 = e1 == hipSuccess ? hipStreamWaitEvent(home, c->joins[k], 0) : e1;
      if (e2 != hipSuccess && rc == DF_OK) rc = hip_fail(c, e2, "join");
    }
  }
  c->stream = home;
  c->ws = ws;
  c->ws_bytes = ws_bytes;
  c->slices = saved_s;
  c->ev_cap = saved_cap;
  c->scr_mask = saved_mask;
  c->scr_chunks = saved_chunks;
  c->scr_blk = saved_blk;
  c->scr_nao = saved_nao;
  return rc;
}

int df_peak_probe(df_ctx* c, int kind, void* buf, size_t bytes, int iters, double* rate) {
  clear_stale_error();
  if (!c) return DF_EINVAL;
  if (kind < 0 || kind > 3 || !buf || !rate) return fail(c, DF_EINVAL, "bad kind, buffer or rate");
  if (reinterpret_cast<uintptr_t>(buf) & 255) return fail(c, DF_EINVAL, "buffer must be 256-byte aligned");
  if (iters < 1 || iters > 1000000) return fail(c, DF_EINVAL, "iters must be 1..10^6");
  const size_t need = kind <= 1 ? (size_t)c->ncu * 8 * 256 * 8 : (size_t)1 << 22;
  if (bytes < need) return fail(c, DF_EINVAL, "buffer too small for this probe");
  hipEvent_t e0, e1;
  DF_HIP(hipEventCreate(&e0), "hipEventCreate");
  hipError_t e = hipEventCreate(&e1);
  if (e != hipSuccess) {
    (void)hipEventDestroy(e0);
    return hip_fail(c, e, "hipEventCreate");
  }
  double work = 0.0;
  constexpr int kReps = 3;
  e = launch_peak(c->stream, kind, c->ncu, buf, bytes, iters, &work);  // warm-up
  if (e == hipSuccess) e = hipEventRecord(e0, c->stream);
  for (int r = 0; r < kReps && e == hipSuccess; ++r)
    e = launch_peak(c->stream, kind, c->ncu, buf, bytes, iters, &work);
  if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return hip_fail(c, e, "peak probe");
  // TOP/s, TFLOP/s or GB/s
  *rate = kind <= 1 ? work * kReps / (ms * 1e-3) / 1e12 : work * kReps / (ms * 1e-3) / 1e9;
  return DF_OK;
}

int df_timing_begin(df_ctx* c, int max_calls) {
  clear_stale_error();
  if (!c) return DF_EINVAL;
  if (max_calls < 1 || max_calls > 100000) return fail(c, DF_EINVAL, "max_calls must be 1..100000");
  for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
  c->ev.assign((size_t)max_calls * (DF_NSTAGES + 1), nullptr);
  for (auto& e : c->ev) {
    const hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) {
      c->ev_cap = 0;
      return hip_fail(c, r, "hipEventCreate");
    }
  }
  c->ev_cap = max_calls;
  c->ev_used = 0;
  return DF_OK;
}

int df_timing_end(df_ctx* c, double* ms_sum, int* ncalls) {
  if (!c) return DF_EINVAL;
  if (!ms_sum || !ncalls) return fail(c, DF_EINVAL, "null output");
  for (int i = 0; i < DF_NSTAGES; ++i) ms_sum[i] = 0.0;
  *ncalls = c->ev_used;
  hipError_t r = hipStreamSynchronize(c->stream);
  if (r != hipSuccess) return hip_fail(c, r, "timing sync");
  for (int call = 0; call < c->ev_used; ++call) {
    hipEvent_t* e = &c->ev[(size_t)call * (DF_NSTAGES + 1)];
    for (int i = 0; i < DF_NSTAGES; ++i) {
      float ms = 0.f;
      r = hipEventElapsedTime(&ms, e[i], e[i + 1]);
      if (r != hipSuccess) return hip_fail(c, r, "hipEventElapsedTime");
      ms_sum[i] += ms;
    }
  }
  for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
  c->ev.clear();
  c->ev_cap = c->ev_used = 0;
  return DF_OK;
}

int df_metric_cholesky(df_ctx* c, double* W, int64_t n) {
  clear_stale_error();
  if (!c) return DF_EINVAL;
  if (!W || n < 1 || n > 65536) return fail(c, DF_EINVAL, "bad W or n");
  DF_HIP(launch_cholesky(c->stream, W, n, c->status), "cholesky");
  return DF_OK;
}

int df_whiten(df_ctx* c, const double* L, int64_t naux, const double* T, int64_t ncols, double* B) {
  clear_stale_error();
  if (!c) return DF_EINVAL;
  if (!L || !T || !B || naux < 1 || naux > 65536 || ncols < 1) return fail(c, DF_EINVAL, "bad arguments");
  if (B == T) return fail(c, DF_EINVAL, "B must not alias T");
  const size_t need = (size_t)naux * naux * 8;
  if (!c->ws || c->ws_bytes < need) return fail(c, DF_EWORKSPACE, "workspace too small for L^-1");
  double* Linv = at<double>(c, 0);
  DF_HIP(launch_tri_inverse(c->stream, L, naux, Linv), "tri_inverse");
  DF_HIP(launch_whiten(c->stream, Linv, naux, T, ncols, B), "whiten");
  return DF_OK;
}

int df_density(df_ctx* c, const double* C, int64_t nao, int64_t nocc, double occ, double* D) {
  clear_stale_error();
  if (!c) return DF_EINVAL;
  if (!C || !D || nao < 1 || nocc < 1 || nocc > nao) return fail(c, DF_EINVAL, "bad arguments");
  DF_HIP(launch_density(c->stream, C, nao, nocc, occ, D), "density");
  return DF_OK;
}

int df_fock(df_ctx* c, const double* h, const double* J, const double* K, const double* D,
            int64_t nao, double* F, double* e_one) {
  clear_stale_error();
  if (!c) return DF_EINVAL;
  if (!h || !J || !K || !D || !F || !e_one || nao < 1 || nao > 65536)
    return fail(c, DF_EINVAL, "bad arguments");
  DF_HIP(launch_fock(c->stream, h, J, K, D, nao, F, reinterpret_cast<double*>(c->aux), e_one),
         "fock");
  return DF_OK;
}

int df_rule_level(double de_rel) {
  if (de_rel != de_rel) return 4;
  if (de_rel >= 2e-6) return 4;
  if (de_rel >= 5e-9) return 3;
  if (de_rel >= 2e-11) return 2;
  if (de_rel >= 7e-14) return 1;
  return 0;
}

int df_rule_next_level(int level, double e_prev, double e_now) {
  const double de = e_now - e_prev;
  const double rel = e_now == 0.0 ? fabs(de) : fabs(de / e_now);
  const int l = df_rule_level(rel);
  return l < level ? l : level;
}

int df_rule_slices(int level, int fp64_below_level) {
  if (level <= 0 || level <= fp64_below_level) return 0;
  static const int mbits[5] = {0, 47, 39, 31, 23};
  const int m = mbits[level > 4 ? 4 : level];
  return (m + 1 + 7) / 8;
}

int df_controller_allocate(const float* pred, int64_t nblocks, int s_ref, double slack,
                           const double* cost, int32_t* s_out) {
  if (!pred || !s_out || nblocks < 1 || s_ref < 0 || s_ref > kMaxSlices || !(slack > 0.0))
    return DF_EINVAL;
  double cs[kMaxSlices];
  for (int k = 0; k < kMaxSlices; ++k) {
    cs[k] = cost ? cost[k] : (double)((k + 1) * (k + 2) / 2);
    if (!std::isfinite(cs[k])) return DF_EINVAL;
  }
  if (s_ref == 0) {
    for (int64_t b = 0; b < nblocks; ++b) s_out[b] = 0;
    return DF_OK;
  }
  // predicted errors, made non-increasing in s
  std::vector<double> err((size_t)nblocks * kMaxSlices);
  for (int64_t b = 0; b < nblocks; ++b) {
    double e = pow(10.0, (double)pred[b * kMaxSlices]);
    for (int k = 0; k < kMaxSlices; ++k) {
      e = std::min(e, pow(10.0, (double)pred[b * kMaxSlices + k]));
      err[b * kMaxSlices + k] = e;
    }
  }
  auto E = [&](int64_t b, int s) { return err[b * kMaxSlices + s - 1]; };
  double budget = 0.0;
  for (int64_t b = 0; b < nblocks; ++b) {
    budget += E(b, s_ref);
    s_out[b] = 1;
  }
  budget *= slack;
  for (;;) {
    double total = 0.0;  // the predicted total, in block order
    for (int64_t b = 0; b < nblocks; ++b) total += E(b, s_out[b]);
    if (!(total > budget)) break;
    // the move with the largest error drop per added cost; a move that adds
    // no cost beats every other (the largest drop first among them)
    int64_t best = -1;
    int best_to = 0;
    bool best_free = false;
    double gain = 0.0;
    for (int64_t b = 0; b < nblocks; ++b) {
      const int sb = s_out[b];
      int to = sb + 1;
      while (to <= kMaxSlices && !(E(b, to) < E(b, sb))) ++to;
      if (to > kMaxSlices) continue;
      const double drop = E(b, sb) - E(b, to);
      const double dc = cs[to - 1] - cs[sb - 1];
      const bool free = !(dc > 0.0);
      const double g = free ? drop : drop / dc;
      if (best < 0 || (free && !best_free) || (free == best_free && g > gain)) {
        best = b;
        best_free = free;
        gain = g;
        best_to = to;
      }
    }
    if (best < 0) break;
    s_out[best] = best_to;
  }
  // then every block takes the largest count that costs no more than its own
  for (int64_t b = 0; b < nblocks; ++b)
    for (int to = kMaxSlices; to > s_out[b]; --to)
      if (!(cs[to - 1] > cs[s_out[b] - 1])) {
        s_out[b] = to;
        break;
      }
  return DF_OK;
}

int df_get_status(df_ctx* c) {
  clear_stale_error();
  if (!c) return DF_EINVAL;
  int h = 0;
  hipError_t e = hipMemcpyAsync(&h, c->status, sizeof(int), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "status read");
  e = launch_fill_i32(c->stream, c->status, 1, 0);
  if (e != hipSuccess) return hip_fail(c, e, "status clear");
  if (h & kStatusNonFinite) return DF_ENONFINITE;
  if (h & kStatusNotSpd) return DF_ENOTSPD;
  return DF_OK;
}

const char* df_last_error(const df_ctx* c) { return c ? c->err.c_str() : "null context"; }

int df_debug_build_i32(df_ctx* c, const double* B, int layout, int64_t naux, int64_t nao,
                       const int32_t* b_exp, const double* C, int64_t nocc, int32_t* x_sums,
                       int32_t* k_sums) {
  clear_stale_error();
  Plan p;
  int rc = common_checks(c, B, layout, naux, nao, C, nocc, p);
  if (rc) return rc;
  if (!x_sums || !k_sums) return fail(c, DF_EINVAL, "null output");
  if (!c->blk_s.empty()) return fail(c, DF_EINVAL, "the export uses one slice count: reset block precision");
  const int s = c->slices;
  if (s < 1) return fail(c, DF_EINVAL, "the export needs 1..8 slices");
  hipStream_t st = c->stream;
  if (!b_exp) {
    int32_t* be = at<int32_t>(c, p.off_bexp);
    DF_HIP(launch_bexp(c, B, p.packed, naux, nao, be), "row_exp");
    b_exp = be;
  }
  double* X = at<double>(c, p.off_X);
  int32_t* fcol = at<int32_t>(c, p.off_fcol);
  int8_t* dC = at<int8_t>(c, p.off_dC);
  unsigned long long* xmax = at<unsigned long long>(c, p.off_xmax);
  DF_HIP(launch_fill_u64(st, xmax, (int64_t)p.nb * p.nao, 0ull), "fill xmax");
  DF_HIP(launch_col_exp(st, C, nao, nocc, fcol, c->status), "col_exp");
  DF_HIP(launch_slice_c(st, C, nao, nocc, s, fcol, p.ncp, p.kp, 0, dC), "slice_c");
  DF_HIP(launch_x_int8(st, s, B, naux, (int)nao, b_exp, dC, p.ncp, p.kp, fcol, (int)nocc, X, 1,
                       xmax, p.pblk, nullptr, nullptr, chunks_for(c, nao),
                       ksub_for(c, naux, nao, nocc), x_sums, p.packed, c->extra),
         "x_int8");
  int32_t* F = at<int32_t>(c, p.off_F);
  int8_t* Xd = at<int8_t>(c, p.off_Xd);
  DF_HIP(launch_slice_x(st, s, X, naux, (int)nao, (int)nocc, p.pblk, p.nao_pad, p.kbp, xmax, F, Xd),
         "slice_x");
  set_xstats(c, p, false);
  DF_HIP(launch_k_int8(st, s, Xd, F, p.nb, (int)nao, p.nao_pad, p.kbp, p.groups,
                       at<double>(c, p.off_Kp), k_sums, c->extra),
         "k_int8");
  return DF_OK;
}

int df_debug_slice_gemm_i32(df_ctx* c, const int8_t* a_dig, const int8_t* b_dig, int64_t m,
                            int64_t n, int64_t k, int s, int32_t* partials) {
  clear_stale_error();
  if (!c) return DF_EINVAL;
  if (!a_dig || !b_dig || !partials) return fail(c, DF_EINVAL, "null pointer");
  if (m < 1 || n < 1 || k < 1 || s < 1 || s > kMaxSlices) return fail(c, DF_EINVAL, "bad shape");
  if (k >= 131072) return fail(c, DF_EOVERFLOW_GUARD, "k >= 131072: 128^2 k reaches 2^31");
  const int64_t mp = round_up(m, 64), np = round_up(n, 64), kpd = round_up(k, 64);
  const size_t need_a = (size_t)s * mp * kpd, need_b = (size_t)s * np * kpd;
  const size_t need = (need_a + 255) / 256 * 256 + need_b;
  if (!c->ws || c->ws_bytes < need) return fail(c, DF_EWORKSPACE, "workspace too small");
  int8_t* wa = at<int8_t>(c, 0);
  int8_t* wb = at<int8_t>(c, (need_a + 255) / 256 * 256);
  DF_HIP(launch_debug_pairs(c->stream, s, a_dig, b_dig, m, n, k, wa, wb, partials), "debug_pairs");
  return DF_OK;
}

}  // extern "C"
