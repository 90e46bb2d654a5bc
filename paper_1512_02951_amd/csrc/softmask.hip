// Differentiation form: a soft per-frequency selection mask m = sigmoid(l)
// over the 64 natural DCT frequencies, the public image it leaves,
//   P = IDCT( DCT(x) * (1 - m) )   per 8x8 block
// (the hard-mask case is the zero-padded public image of the report,
// Sec. 6.3.1 / Fig. 7b), and its hand-written adjoint:
//   dL/dm_n = - sum over images and blocks of DCT(dL/dP)_n * DCT(x)_n,
// the transposed (= inverse, the basis being orthonormal) transform applied to
// the upstream gradient.  The objective used to tune the mask is the mean
// squared Pearson correlation (Sec. 6.6.2) between P and x per image plus a
// budget penalty lam * (sum m - budget)^2.
//
// Kernels (one 8x8 block per lane, tiles of 64 blocks inside one image):
//   sm_forward      x -> P (optional) and per-workgroup partial sums of
//                   E_n = sum over blocks of DCT(x)_n^2 and sum x
//   sm_stats        (x, P) -> partial sums of x, P, xP, x^2, P^2
//   sm_backward     (x, G) -> partial sums of DCT(G)_n DCT(x)_n
//   sm_reduce       deterministic FP64 reduction of the partials
//   sm_loss         image statistics -> loss, per-image gradient
//                   coefficients, closed-form dL/dl (Parseval), budget term
//   sm_corr_grad    G = a (x - mean x) + b (P - mean P), scaled
// Partial sums are FP32 within a lane, then FP64 across lanes and workgroups.
#include "plain_tile.h"

namespace sf {
namespace {

constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;
constexpr int kStats = 65;     // E_0 .. E_63, sum x
constexpr int kCorrStats = 5;  // sum x, sum P, sum xP, sum x^2, sum P^2
constexpr uint64_t kTuneStatsLdsBytes = 48u * 1024u;

struct SmGeom {
  uint32_t B, H, W, Bx;
  uint32_t blocks;       // per image
  uint32_t tiles;        // per image
  uint32_t wg_per_image; // grid.x
};

__host__ __device__ inline SmGeom sm_geom(uint32_t B, uint32_t H, uint32_t W, uint32_t num_cu) {
  SmGeom g;
  g.B = B;
  g.H = H;
  g.W = W;
  g.Bx = W / 8;
  g.blocks = (H / 8) * (W / 8);
  g.tiles = (g.blocks + 63) / 64;
  // enough workgroups to cover every CU about twice, at most one wave per tile
  // (more workgroups measured slower, also for the statistics-only pass,
  // whose registers would allow them)
  uint32_t want = (2 * num_cu + B - 1) / B;
  const uint32_t cap = (g.tiles + kWaves - 1) / kWaves;
  g.wg_per_image = want < 1 ? 1 : (want > cap ? cap : want);
  return g;
}

// Loads the lane's 8x8 block of a float image (row-major plane) into c[8y + x].
__device__ __forceinline__ void load_fblock(const float *plane, uint32_t W, uint32_t org, bool valid, float (&c)[64]) {
  if (valid) {
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const float4 a = *reinterpret_cast<const float4 *>(plane + org + (size_t)r * W);
      const float4 b = *reinterpret_cast<const float4 *>(plane + org + (size_t)r * W + 4);
      c[8 * r + 0] = a.x;
      c[8 * r + 1] = a.y;
      c[8 * r + 2] = a.z;
      c[8 * r + 3] = a.w;
      c[8 * r + 4] = b.x;
      c[8 * r + 5] = b.y;
      c[8 * r + 6] = b.z;
      c[8 * r + 7] = b.w;
    }
  } else {
#pragma unroll
    for (int p = 0; p < 64; ++p) c[p] = 0.0f;
  }
}

// P is written once per call: streaming (non-temporal) stores (measured 9 %
// faster for the forward with P than default-policy stores; non-temporal
// loads of x were slower).
typedef float f4v __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void store_fblock(float *plane, uint32_t W, uint32_t org, const float (&c)[64]) {
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const f4v a = {c[8 * r], c[8 * r + 1], c[8 * r + 2], c[8 * r + 3]};
    const f4v b = {c[8 * r + 4], c[8 * r + 5], c[8 * r + 6], c[8 * r + 7]};
    __builtin_nontemporal_store(a, reinterpret_cast<f4v *>(plane + org + (size_t)r * W));
    __builtin_nontemporal_store(b, reinterpret_cast<f4v *>(plane + org + (size_t)r * W + 4));
  }
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

__device__ __forceinline__ void swap_halves(float &a, float &b, bool rows16) {
  const auto r = rows16 ? __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false)
                        : __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  a = __uint_as_float(r[0]);
  b = __uint_as_float(r[1]);
}

// Wave reduce-scatter by recursive halving: val(n) is the lane's value for
// frequency n; returns, in lane L, the sum over the wave's 64 lanes of their
// values for frequency L (63 exchanges instead of 64 x 6 for 64 wave sums).
// Steps 32 and 16 pair lanes with v_permlane32_swap / v_permlane16_swap (the
// swapped operands land so that one add finishes the step), steps 8..1 with
// xor shuffles and a select of the half each lane keeps.  The values are
// formed pairwise inside the first step, so at most 32 partial sums are live.
template <class F>
__device__ __forceinline__ float wave_reduce_scatter(F &&val) {
  const int lane = threadIdx.x & 63;
  float h[32];
#pragma unroll
  for (int j = 0; j < 32; ++j) {
    float lo = val(j), hi = val(32 + j);
    swap_halves(lo, hi, false);
    h[j] = lo + hi;
  }
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    swap_halves(h[j], h[16 + j], true);
    h[j] += h[16 + j];
  }
  static_for<0, 4>([&](auto sc) {
    constexpr int d = 8 >> decltype(sc)::value;
    const bool up = lane & d;
    static_for<0, d>([&](auto jc) {
      constexpr int j = decltype(jc)::value;
      const float keep = up ? h[d + j] : h[j], send = up ? h[j] : h[d + j];
      h[j] = keep + __shfl_xor(send, d, 64);
    });
  });
  return h[0];
}

// Workgroup loop: tiles t = blockIdx.x * kWaves + wave + i * stride of image
// blockIdx.y; body(org, valid) per tile.
template <class Body>
__device__ __forceinline__ void sm_tiles(const SmGeom &g, Body &&body) {
  const int lane = threadIdx.x & 63;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint32_t stride = gridDim.x * kWaves;
  for (uint32_t t = blockIdx.x * kWaves + wave; t < g.tiles; t += stride) {
    const uint32_t blk = t * 64u + (uint32_t)lane;
    const bool valid = blk < g.blocks;
    const uint32_t by = blk / g.Bx, bx = blk - by * g.Bx;
    const uint32_t org = valid ? by * 8u * g.W + bx * 8u : 0u;
    body(org, valid);
  }
}

// Writes the workgroup's kN sums as FP64 partials to
// out[(image * wg_per_image + blockIdx.x) * kN + k].  Sums k < kLane come one
// per lane (lane k holds the wave's total for k, already reduced across the
// wave); the kN - kLane others are per-lane values still to be wave-summed.
template <int kN, int kLane>
__device__ __forceinline__ void wg_partials(float lane_val, const float *rest, double *out,
                                            const SmGeom &g) {
  __shared__ double s[kWaves][kN];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (kLane > 0 && lane < kLane) s[wave][lane] = (double)lane_val;
#pragma unroll
  for (int k = 0; k < kN - kLane; ++k) {
    const float w = wave_sum(rest[k]);
    if (lane == 0) s[wave][kLane + k] = (double)w;
  }
  __syncthreads();
  double *dst = out + ((size_t)blockIdx.y * g.wg_per_image + blockIdx.x) * kN;
  for (int k = threadIdx.x; k < kN; k += kThreads) {
    double v = 0.0;
    for (int w = 0; w < kWaves; ++w) v += s[w][k];
    dst[k] = v;
  }
}

struct SmArgs {
  SmGeom g;
  const float *x;
  const float *y;     // P (stats) or G (backward)
  float *p_out;       // forward: P (may be null)
  const float *logits;
  double *partials;
  DctK K;
};

// Statistics per image: E_0 .. E_63, then sum x; with kP also P.  Two
// instantiations so that the statistics-only pass is not held to the
// registers of the pass that keeps the coefficients for P.
template <bool kP>
__global__ __launch_bounds__(kThreads) void sm_forward_kernel(SmArgs a) {
  __shared__ float s_keep[64];
  if (threadIdx.x < 64) s_keep[threadIdx.x] = 1.0f - 1.0f / (1.0f + __expf(-a.logits[threadIdx.x]));
  __syncthreads();
  const SmGeom &g = a.g;
  const size_t plane = (size_t)blockIdx.y * g.H * g.W;
  float e_acc = 0.0f;   // lane n: energy of frequency n over the wave's blocks
  float sx[1] = {0.0f}; // per lane: sum of its blocks' samples
  __shared__ f4v s_rows[kP ? kWaves : 1][128];  // per wave: one row of P for 64 blocks
  f4v *srow = s_rows[kP ? threadIdx.x >> 6 : 0];
  const bool rows = kP && g.Bx % 64u == 0u;   // every tile: 64 consecutive blocks of one block row
  sm_tiles(g, [&](uint32_t org, bool valid) {
    float c[64];
    load_fblock(a.x + plane, g.W, org, valid, c);
    float s = 0.0f;
#pragma unroll
    for (int p = 0; p < 64; ++p) s += c[p];
    sx[0] += s;
    fdct8x8(c, a.K);
    e_acc += wave_reduce_scatter([&](int n) { return c[n] * c[n]; });
    if constexpr (kP) {
      const float *keep = s_keep + opaque_zero();  // re-read per tile: not 64 live registers
#pragma unroll
      for (int n = 0; n < 64; ++n) c[n] *= keep[n];
      idct8x8(c, a.K);
      if (rows) {
        // each row of the tile through LDS, so that one store instruction
        // writes 1 KB of contiguous samples (32 blocks' row segments, whole
        // cache lines) instead of every other 16 bytes of 2 KB
        const uint32_t lane = threadIdx.x & 63u;
        float *dst = a.p_out + plane + __builtin_amdgcn_readfirstlane(org);
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          const f4v lo = {c[8 * r], c[8 * r + 1], c[8 * r + 2], c[8 * r + 3]};
          const f4v hi = {c[8 * r + 4], c[8 * r + 5], c[8 * r + 6], c[8 * r + 7]};
          srow[2 * lane] = lo;
          srow[2 * lane + 1] = hi;
          const f4v v0 = srow[lane], v1 = srow[64 + lane];
          __builtin_nontemporal_store(v0, reinterpret_cast<f4v *>(dst + (size_t)r * g.W + 4u * lane));
          __builtin_nontemporal_store(v1, reinterpret_cast<f4v *>(dst + (size_t)r * g.W + 256u + 4u * lane));
        }
      } else if (valid) {
        store_fblock(a.p_out + plane, g.W, org, c);
      }
    }
  });
  wg_partials<kStats, 64>(e_acc, sx, a.partials, g);
}

__global__ __launch_bounds__(kThreads) void sm_stats_kernel(SmArgs a) {
  const SmGeom &g = a.g;
  const size_t plane = (size_t)blockIdx.y * g.H * g.W;
  float acc[kCorrStats] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
  sm_tiles(g, [&](uint32_t org, bool valid) {
    if (!valid) return;
#pragma unroll
    for (int r = 0; r < 8; ++r)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const float4 xv = *reinterpret_cast<const float4 *>(a.x + plane + org + (size_t)r * g.W + 4 * h);
        const float4 pv = *reinterpret_cast<const float4 *>(a.y + plane + org + (size_t)r * g.W + 4 * h);
        const float xs[4] = {xv.x, xv.y, xv.z, xv.w}, ps[4] = {pv.x, pv.y, pv.z, pv.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          acc[0] += xs[i];
          acc[1] += ps[i];
          acc[2] = __builtin_fmaf(xs[i], ps[i], acc[2]);
          acc[3] = __builtin_fmaf(xs[i], xs[i], acc[3]);
          acc[4] = __builtin_fmaf(ps[i], ps[i], acc[4]);
        }
      }
  });
  wg_partials<kCorrStats, 0>(0.0f, acc, a.partials, g);
}

__global__ __launch_bounds__(kThreads) void sm_backward_kernel(SmArgs a) {
  const SmGeom &g = a.g;
  const size_t plane = (size_t)blockIdx.y * g.H * g.W;
  float acc = 0.0f;  // lane n: sum of DCT(G)_n DCT(x)_n over the wave's blocks
  sm_tiles(g, [&](uint32_t org, bool valid) {
    float cx[64], cg[64];
    load_fblock(a.x + plane, g.W, org, valid, cx);
    fdct8x8(cx, a.K);
    load_fblock(a.y + plane, g.W, org, valid, cg);
    fdct8x8(cg, a.K);  // adjoint of the inverse transform
    acc += wave_reduce_scatter([&](int n) { return cg[n] * cx[n]; });
  });
  wg_partials<64, 64>(acc, nullptr, a.partials, g);
}

// out[i * kN + k] = sum over parts of partials[(i * parts + j) * kN + k], j in order.
__global__ void sm_reduce_kernel(const double *partials, uint32_t items, uint32_t parts, uint32_t kN, double *out) {
  const uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= items * kN) return;
  const uint32_t i = idx / kN, k = idx - i * kN;
  double s = 0.0;
  for (uint32_t j = 0; j < parts; ++j) s += partials[((size_t)i * parts + j) * kN + k];
  out[idx] = s;
}

struct LossArgs {
  const double *stats;     // B x 65 (closed form) or B x 5 (corr) per mode
  uint32_t B;
  double N;                // samples per image
  double inv_n;            // 1 / N
  double lam, budget;
  int mode;                // 0: closed form from B x 65 energies; 1: from B x 5 correlation sums
  float *gcoef;            // B x 4: a, b, mean x, mean P of dL/dP, or null
};

struct LossShared {
  double m[64];
  double alpha[256], beta[256], dc[256];  // per image, in chunks of 256
};

// Objective at mask m_n = sigmoid(l) for the calling thread's frequency
// n = threadIdx.x (64 threads, one wave).  Returns the loss in every thread and
// sets dm to dL/dm_n of the correlation part (mode 0 only; zero in mode 1) and
// gb to the budget part 2 lam (sum m - budget), m_out to m_n.  Per image b (population
// moments over the N samples):
//   rho_b = cov(P, x) / (sd x sd P),
//   dL/dP = a_b (x - mean x) + b_b (P - mean P),
//   a_b = 2 rho_b / (B N sd x sd P),  b_b = -2 rho_b^2 / (B N var P).
// Mode 0 takes the moments of P from the energies by Parseval: with
// keep_n = 1 - m_n, sum xP = sum_n keep_n E_n, sum P^2 = sum_n keep_n^2 E_n,
// sum x^2 = sum_n E_n, mean P = keep_0 mean x (only the DC basis function has
// a nonzero mean), and dL/dm_n = -sum_b (a_b dE'_bn + b_b keep_n dE'_bn) with
// the DC term corrected for the means.
// Sum over the wave in a fixed order (a shift-down tree into lane 0, then
// lane 0's value to every lane): the same bits in every lane and every call.
__device__ __forceinline__ double wave_sum_fixed(double v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_down(v, d, 64);
  return __shfl(v, 0, 64);
}

__device__ double sm_eval(const LossArgs &a, double l, LossShared &S, double &dm, double &gb, double &m_out) {
  const int n = threadIdx.x;
  const double m = 1.0 / (1.0 + exp(-l));
  m_out = m;
  S.m[n] = m;
  const double msum = wave_sum_fixed(m);
  __syncthreads();
  const double keep0 = 1.0 - S.m[0];
  const double keep_n = 1.0 - m;
  double r2 = 0.0;  // this thread's images, in image order
  // four independent partial sums over the images (image i into i % 4) keep
  // the loop from waiting on one long chain of dependent adds
  double dmp[4] = {0.0, 0.0, 0.0, 0.0};
  for (uint32_t b0 = 0; b0 < a.B; b0 += 256) {
    const uint32_t nb = a.B - b0 < 256 ? a.B - b0 : 256;
    for (uint32_t i = n; i < nb; i += 64) {
      const uint32_t b = b0 + i;
      double sx, sp, sxp, sxx, spp;
      if (a.mode == 0) {
        const double *st = a.stats + (size_t)b * kStats;
        sx = st[64];
        sxx = 0.0;
        sxp = 0.0;
        spp = 0.0;
#pragma unroll 8
        for (int k = 0; k < 64; ++k) {
          const double keep = 1.0 - S.m[k], e = st[k];
          sxx += e;
          sxp += keep * e;
          spp += keep * keep * e;
        }
        sp = keep0 * sx;
      } else {
        const double *st = a.stats + (size_t)b * kCorrStats;
        sx = st[0];
        sp = st[1];
        sxp = st[2];
        sxx = st[3];
        spp = st[4];
      }
      const double N = a.N, iN = a.inv_n;
      const double xm = sx * iN, pm = sp * iN;
      const double cov = sxp * iN - xm * pm, vx = sxx * iN - xm * xm, vp = spp * iN - pm * pm;
      const double sdx = sqrt(vx > 0 ? vx : 0.0), sdp = sqrt(vp > 1e-300 ? vp : 1e-300);
      const double rho = cov / (sdx * sdp + 1e-300);
      const double alpha = 2.0 * rho / ((double)a.B * N * sdx * sdp + 1e-300);
      const double beta = -2.0 * rho * rho / ((double)a.B * N * vp + 1e-300);
      S.alpha[i] = alpha;
      S.beta[i] = beta;
      // the DC term's correction for the means, once per image
      S.dc[i] = alpha * N * xm * xm + beta * N * pm * xm;
      r2 += rho * rho;
      if (a.gcoef) {
        a.gcoef[4 * b + 0] = (float)alpha;
        a.gcoef[4 * b + 1] = (float)beta;
        a.gcoef[4 * b + 2] = (float)xm;
        a.gcoef[4 * b + 3] = (float)pm;
      }
    }
    __syncthreads();
    if (a.mode == 0) {
#pragma unroll 4
      for (uint32_t i = 0; i < nb; ++i) {
        const double E = a.stats[(size_t)(b0 + i) * kStats + n];
        double t = S.alpha[i] * E + S.beta[i] * keep_n * E;
        if (n == 0) t -= S.dc[i];
        dmp[i & 3] -= t;
      }
    }
    __syncthreads();
  }
  dm = (dmp[0] + dmp[1]) + (dmp[2] + dmp[3]);
  const double rho2 = wave_sum_fixed(r2);
  const double over = msum - a.budget;
  gb = 2.0 * a.lam * over;
  return rho2 / (double)a.B + a.lam * over * over;
}

// One evaluation: loss, closed-form gradient (mode 0), budget gradient and
// the per-image coefficients of dL/dP.
__global__ __launch_bounds__(64) void sm_loss_kernel(LossArgs a, const float *logits, double *loss, float *grad_logits,
                                                     float *grad_budget) {
  __shared__ LossShared S;
  const int n = threadIdx.x;
  double dm, gb, m;
  const double l = (double)logits[n];
  const double L = sm_eval(a, l, S, dm, gb, m);
  const double sig = m * (1.0 - m);
  if (grad_logits) grad_logits[n] = (float)(sig * (dm + gb));
  if (grad_budget) grad_budget[n] = (float)(sig * gb);
  if (n == 0) loss[0] = L;
}

// The whole tuning loop on fixed statistics: Adam on the 64 logits
// (beta1 0.9, beta2 0.999, eps 1e-8), loss before each step into trace, then
// the n_private largest logits (ties to the lower frequency) hardened into a
// private_mask: bit z set for the zigzag position z of each chosen frequency.
// stats_lds: number of statistics doubles staged in LDS (dynamic shared
// memory) for the whole loop, or 0 to read them from global memory each step.
__global__ __launch_bounds__(64) void sm_tune_kernel(LossArgs a, float *logits, uint32_t steps, double lr,
                                                     double *trace, uint64_t *mask_out, uint32_t n_private,
                                                     uint32_t stats_lds) {
  __shared__ LossShared S;
  __shared__ double s_l[64];
  extern __shared__ double s_stats[];
  const int n = threadIdx.x;
  if (stats_lds) {
    for (uint32_t i = n; i < stats_lds; i += 64) s_stats[i] = a.stats[i];
    __syncthreads();
    a.stats = s_stats;
  }
  double l = (double)logits[n], mom = 0.0, vel = 0.0, p1 = 1.0, p2 = 1.0;
  for (uint32_t t = 0; t < steps; ++t) {
    double dm, gb, m;
    const double L = sm_eval(a, l, S, dm, gb, m);
    if (trace && n == 0) trace[t] = L;
    const double g = m * (1.0 - m) * (dm + gb);
    mom = 0.9 * mom + 0.1 * g;
    vel = 0.999 * vel + 0.001 * g * g;
    p1 *= 0.9;
    p2 *= 0.999;
    l -= lr * (mom / (1.0 - p1)) / (sqrt(vel / (1.0 - p2)) + 1e-8);
  }
  logits[n] = (float)l;
  s_l[n] = (double)(float)l;
  __syncthreads();
  uint32_t rank = 0;
  for (int k = 0; k < 64; ++k) rank += (s_l[k] > s_l[n]) || (s_l[k] == s_l[n] && k < n);
  // lane z of the ballot asks whether the frequency at zigzag position z is chosen
  __shared__ uint32_t s_sel[64];
  s_sel[kZigZagInv.pos[n]] = rank < n_private ? 1u : 0u;
  __syncthreads();
  const uint64_t bits = __ballot(s_sel[n] != 0u);
  if (mask_out && n == 0) mask_out[0] = bits;
}

// G = scale * (a_b (x - xm_b) + b_b (P - pm_b)), elementwise; scale = *d_scale
// (1 if null).  Block 0 also writes grad_out[n] = scale * grad_budget[n].
__global__ void sm_corr_grad_kernel(const float *x, const float *p, const float *gcoef, const double *d_scale, float *g,
                                    uint32_t B, uint64_t per_image, const float *grad_budget, float *grad_out) {
  const float scale = d_scale ? (float)d_scale[0] : 1.0f;
  if (blockIdx.x == 0 && threadIdx.x < 64 && grad_budget && grad_out)
    grad_out[threadIdx.x] = scale * grad_budget[threadIdx.x];
  const uint64_t n = (uint64_t)B * per_image;
  for (uint64_t i = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4; i < n;
       i += (uint64_t)gridDim.x * blockDim.x * 4) {
    const uint32_t b = (uint32_t)(i / per_image);
    const float al = gcoef[4 * b] * scale, be = gcoef[4 * b + 1] * scale, xm = gcoef[4 * b + 2], pm = gcoef[4 * b + 3];
    const float4 xv = *reinterpret_cast<const float4 *>(x + i);
    const float4 pv = *reinterpret_cast<const float4 *>(p + i);
    float4 o;
    o.x = __builtin_fmaf(al, xv.x - xm, be * (pv.x - pm));
    o.y = __builtin_fmaf(al, xv.y - xm, be * (pv.y - pm));
    o.z = __builtin_fmaf(al, xv.z - xm, be * (pv.z - pm));
    o.w = __builtin_fmaf(al, xv.w - xm, be * (pv.w - pm));
    *reinterpret_cast<float4 *>(g + i) = o;
  }
}

// dL/dl_n = sigmoid'(l_n) * dL/dm_n with dL/dm_n = -sum DCT(G)_n DCT(x)_n.
__global__ void sm_adjoint_grad_kernel(const double *adj, const float *logits, float *grad_logits) {
  const int n = threadIdx.x;
  const double m = 1.0 / (1.0 + exp(-(double)logits[n]));
  grad_logits[n] = (float)(m * (1.0 - m) * -adj[n]);
}

int sm_check(uint32_t B, uint32_t H, uint32_t W) {
  if (B == 0 || H == 0 || W == 0 || H % 8 || W % 8) return fail(SF_ESHAPE, "B >= 1 and H, W positive multiples of 8");
  if ((uint64_t)H * W >= (1ull << 32)) return fail(SF_ESHAPE, "image too large");
  return SF_OK;
}

// Many parts per output: one workgroup per output, 256 threads summing
// strided parts in a fixed order, then a fixed LDS tree (deterministic).
__global__ __launch_bounds__(256) void sm_reduce_wide_kernel(const double *partials, uint32_t parts, uint32_t kN,
                                                              double *out) {
  __shared__ double s[256];
  const uint32_t o = blockIdx.x, i = o / kN, k = o - i * kN;
  double v = 0.0;
  for (uint32_t j = threadIdx.x; j < parts; j += 256) v += partials[((size_t)i * parts + j) * kN + k];
  s[threadIdx.x] = v;
  __syncthreads();
  for (uint32_t w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[o] = s[0];
}

int sm_launch_reduce(const double *partials, uint32_t items, uint32_t parts, uint32_t kN, double *out,
                     hipStream_t stream) {
  const uint32_t total = items * kN;
  if (parts > 64)
    hipLaunchKernelGGL(sm_reduce_wide_kernel, dim3(total), dim3(256), 0, stream, partials, parts, kN, out);
  else
    hipLaunchKernelGGL(sm_reduce_kernel, dim3((total + 255) / 256), dim3(256), 0, stream, partials, items, parts,
                       kN, out);
  return SF_OK;
}

}  // namespace

size_t softmask_workspace_bytes(const DeviceState &ds, uint32_t B, uint32_t H, uint32_t W) {
  const SmGeom g = sm_geom(B, H, W, (uint32_t)ds.num_cu);
  return (size_t)B * g.wg_per_image * kStats * sizeof(double) + (size_t)64 * sizeof(double);
}

// Workspace of sf_softmask_forward_noalloc: one copy per device for the life
// of the process.  Host code must not pass this name to a kernel (it is a host
// stand-in, not a device address); it uses the address that
// softmask_scratch_address returns for the current device.
static __device__ __align__(256) uint8_t scratch[kSoftmaskScratchBytes];

int softmask_scratch_address(void **ptr) {
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(soft-mask scratch)");
  *ptr = p;
  return SF_OK;
}

int softmask_forward_noalloc(const DeviceState &ds, const float *x, uint32_t B, uint32_t H, uint32_t W,
                             const float *logits, float *p_out, double *stats, hipStream_t stream) {
  if (int rc = sm_check(B, H, W)) return rc;
  if (!ds.d_sm_scratch) return fail(SF_EHIP, "soft-mask scratch address not initialised");
  // the forward writes every partial slot it later reduces: nothing to clear
  const size_t need = softmask_workspace_bytes(ds, B, H, W);
  if (need > kSoftmaskScratchBytes)
    return fail(SF_ERANGE, "batch too large for the allocation-free forward: needs " + std::to_string(need) +
                               " bytes of partial sums, the static scratch holds " +
                               std::to_string(kSoftmaskScratchBytes));
  return softmask_forward(ds, x, B, H, W, logits, p_out, stats, ds.d_sm_scratch, kSoftmaskScratchBytes, stream);
}

int softmask_forward(const DeviceState &ds, const float *x, uint32_t B, uint32_t H, uint32_t W, const float *logits,
                     float *p_out, double *stats, void *ws, size_t ws_bytes, hipStream_t stream) {
  if (int rc = sm_check(B, H, W)) return rc;
  const SmGeom g = sm_geom(B, H, W, (uint32_t)ds.num_cu);
  if (ws_bytes < softmask_workspace_bytes(ds, B, H, W)) return fail(SF_ERANGE, "soft-mask workspace too small");
  SmArgs a;
  a.g = g;
  a.x = x;
  a.y = nullptr;
  a.p_out = p_out;
  a.logits = logits;
  a.partials = (double *)ws;
  a.K = host_tables().dct;
  if (p_out)
    hipLaunchKernelGGL(sm_forward_kernel<true>, dim3(g.wg_per_image, B), dim3(kThreads), 0, stream, a);
  else
    hipLaunchKernelGGL(sm_forward_kernel<false>, dim3(g.wg_per_image, B), dim3(kThreads), 0, stream, a);
  sm_launch_reduce(a.partials, B, g.wg_per_image, kStats, stats, stream);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SF_OK : hip_fail(e, "soft-mask forward launch");
}

int softmask_corr_stats(const DeviceState &ds, const float *x, const float *p, uint32_t B, uint32_t H, uint32_t W,
                        double *stats, void *ws, size_t ws_bytes, hipStream_t stream) {
  if (int rc = sm_check(B, H, W)) return rc;
  const SmGeom g = sm_geom(B, H, W, (uint32_t)ds.num_cu);
  if (ws_bytes < softmask_workspace_bytes(ds, B, H, W)) return fail(SF_ERANGE, "soft-mask workspace too small");
  SmArgs a{};
  a.g = g;
  a.x = x;
  a.y = p;
  a.partials = (double *)ws;
  a.K = host_tables().dct;
  hipLaunchKernelGGL(sm_stats_kernel, dim3(g.wg_per_image, B), dim3(kThreads), 0, stream, a);
  sm_launch_reduce(a.partials, B, g.wg_per_image, kCorrStats, stats, stream);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SF_OK : hip_fail(e, "soft-mask stats launch");
}

int softmask_backward(const DeviceState &ds, const float *x, const float *gpub, uint32_t B, uint32_t H, uint32_t W,
                      const float *logits, float *grad_logits, void *ws, size_t ws_bytes, hipStream_t stream) {
  if (int rc = sm_check(B, H, W)) return rc;
  const SmGeom g = sm_geom(B, H, W, (uint32_t)ds.num_cu);
  if (ws_bytes < softmask_workspace_bytes(ds, B, H, W)) return fail(SF_ERANGE, "soft-mask workspace too small");
  SmArgs a{};
  a.g = g;
  a.x = x;
  a.y = gpub;
  a.partials = (double *)ws;
  a.K = host_tables().dct;
  hipLaunchKernelGGL(sm_backward_kernel, dim3(g.wg_per_image, B), dim3(kThreads), 0, stream, a);
  // all images and workgroups together: one item of B * wg_per_image parts
  double *adj = (double *)((uint8_t *)ws + (size_t)B * g.wg_per_image * kStats * sizeof(double));
  sm_launch_reduce(a.partials, 1, B * g.wg_per_image, 64, adj, stream);
  hipLaunchKernelGGL(sm_adjoint_grad_kernel, dim3(1), dim3(64), 0, stream, adj, logits, grad_logits);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SF_OK : hip_fail(e, "soft-mask backward launch");
}

static LossArgs loss_args(const double *stats, int mode, uint32_t B, uint32_t H, uint32_t W, float lam, float budget,
                          float *gcoef) {
  LossArgs L{};
  L.stats = stats;
  L.B = B;
  L.N = (double)H * (double)W;
  L.inv_n = 1.0 / L.N;
  L.lam = lam;
  L.budget = budget;
  L.mode = mode;
  L.gcoef = gcoef;
  return L;
}

int softmask_loss(const double *stats, int mode, const float *logits, uint32_t B, uint32_t H, uint32_t W, float lam,
                  float budget, double *loss, float *grad_logits, float *grad_budget, float *gcoef,
                  hipStream_t stream) {
  if (int rc = sm_check(B, H, W)) return rc;
  const LossArgs L = loss_args(stats, mode, B, H, W, lam, budget, gcoef);
  hipLaunchKernelGGL(sm_loss_kernel, dim3(1), dim3(64), 0, stream, L, logits, loss, grad_logits, grad_budget);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SF_OK : hip_fail(e, "soft-mask loss launch");
}

int softmask_tune(const double *stats, uint32_t B, uint32_t H, uint32_t W, float lam, float budget, uint32_t steps,
                  float lr, float *logits, double *trace, uint64_t *mask, uint32_t n_private, hipStream_t stream) {
  if (int rc = sm_check(B, H, W)) return rc;
  if (n_private > 64) return fail(SF_EINVAL, "n_private must be at most 64");
  if (!(lr > 0.0f)) return fail(SF_EINVAL, "learning rate must be positive");
  const LossArgs L = loss_args(stats, 0, B, H, W, lam, budget, nullptr);
  // every step reads all B x 65 statistics: keep them in LDS when they fit
  // beside the static arrays within 64 KB (B <= 94 images)
  const uint64_t nst = (uint64_t)B * kStats;
  const uint32_t stats_lds = nst * sizeof(double) <= kTuneStatsLdsBytes ? (uint32_t)nst : 0u;
  hipLaunchKernelGGL(sm_tune_kernel, dim3(1), dim3(64), (size_t)stats_lds * sizeof(double), stream, L, logits, steps,
                     (double)lr, trace, mask, n_private, stats_lds);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SF_OK : hip_fail(e, "soft-mask tune launch");
}

int softmask_corr_grad(const float *x, const float *p, uint32_t B, uint32_t H, uint32_t W, const float *gcoef,
                       const double *scale, float *g, const float *grad_budget, float *grad_out, hipStream_t stream) {
  if (int rc = sm_check(B, H, W)) return rc;
  const uint64_t n = (uint64_t)B * H * W;
  uint64_t grid = (n / 4 + 255) / 256;
  if (grid > 4096) grid = 4096;
  hipLaunchKernelGGL(sm_corr_grad_kernel, dim3((unsigned)grid), dim3(256), 0, stream, x, p, gcoef, scale, g, B,
                     (uint64_t)H * W, grad_budget, grad_out);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SF_OK : hip_fail(e, "soft-mask correlation gradient launch");
}

}  // namespace sf
