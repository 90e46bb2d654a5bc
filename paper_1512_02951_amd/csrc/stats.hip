// Security statistics of a protected image against its original (report
// Sec. 6.6 and 6.10, Eqs. (3)-(4), Table 14): byte histograms and uniformity,
// entropies and normalised mutual information from the joint histogram,
// block entropy (h = 8), correlation of adjacent samples, two-dimensional
// correlation, bit difference and PSNR.
//
// Three kernels, every moment an exact integer:
//  * band kernel: one wavefront per band of 8 rows x 256 columns of a plane,
//    one 4-sample word per lane and row.  Pair products with v_dot4_u32_u8 on
//    the word and its neighbours (v_alignbyte_b32 shifts in the next lane's
//    first byte): horizontal, vertical and diagonal pairs, sums, squares, the
//    X.Y products and differing bits (v_bcnt).  Pairs that leave the plane
//    multiply a zero; the directional sums of x and y are derived exactly from
//    whole-plane sums minus the border sums the band kernel also gathers.
//    Block entropy: per-wave LDS byte counters (256 per block, four to a
//    word, ds_add), then the product of every sample's value count; H = 6 -
//    log2(product) / 64.  Per-workgroup partial sums.
//  * joint histogram: a workgroup owns the half of the 256 x 256 bins with
//    x < 128 or x >= 128 as 32768 LDS counters (128 KB), counts a chunk of
//    samples, then adds its non-zero bins to the global histogram.
//  * rows (256 workgroups) and finalize (one workgroup): reduce the partials
//    and the histogram in fixed orders, then form the histograms, entropies,
//    NMI, chi-square and correlations in FP64.
#include "sf_internal.h"

namespace sf {
namespace {

constexpr int kBandWaves = 4;
constexpr int kBandThreads = 64 * kBandWaves;
constexpr int kBandGrid = 1024;  // the most band workgroups: one partial slot each
constexpr uint32_t kFlushBands = 256;
constexpr int kJointThreads = 1024;
constexpr uint32_t kHalfBins = 32768;
constexpr int kFinThreads = 256;

// Integer moments of one image gathered by the band kernel.
enum : int {
  kT1 = 0, kT2, kSh, kSv, kSd,    // sum x, sum x^2, horizontal / vertical / diagonal products
  kR0S, kR0Q, kRLS, kRLQ,         // first / last row of each plane: sum, sum of squares
  kC0S, kC0Q, kCLS, kCLQ,         // first / last column
  kTLS, kTLQ, kBRS, kBRQ,         // top-left and bottom-right samples
  kImgMoments
};
constexpr int kCrossXY = 2 * kImgMoments;      // sum x y
constexpr int kBitsDiff = kCrossXY + 1;        // differing bits
constexpr int kIntMoments = kBitsDiff + 1;
// Floating partials: per image sum H, sum H^2, min H, max H.
constexpr int kFltMoments = 8;

struct Partial {
  uint64_t m[kIntMoments];
  double f[kFltMoments];
};

struct StatsGeom {
  uint32_t H, W, C, By, Bx;
  uint32_t wpr;     // words (4 samples) per row = W / 4
  uint32_t nbx;     // bands across a plane = ceil(wpr / 64)
  uint32_t nbands;  // C * By * nbx
};

__device__ __forceinline__ uint32_t udot4(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_udot4(a, b, c, false);
}

__device__ __forceinline__ uint32_t next_bytes(uint32_t w, uint32_t nx) {
  return __builtin_amdgcn_alignbyte(nx, w, 1);  // bytes w1 w2 w3 nx0
}

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// One image's moments over one band; adds into acc.  A band adds at most
// 32 * 255^2 = 2 080 800 to a lane's 32-bit sum; the kernel moves the lane
// sums into the wave's 64-bit record every kFlushBands bands (256 * 2 080 800
// < 2^32), so no image shape can wrap them.
__device__ __forceinline__ void band_image_moments(const uint32_t (&w)[9], const uint32_t (&nx)[9], bool top,
                                                   bool bottom, bool left, bool right, uint32_t *acc) {
  uint32_t t1 = 0, t2 = 0, sh = 0, sv = 0, sd = 0;
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    t1 = udot4(w[r], 0x01010101u, t1);
    t2 = udot4(w[r], w[r], t2);
    sh = udot4(w[r], next_bytes(w[r], nx[r]), sh);
    sv = udot4(w[r], w[r + 1], sv);
    sd = udot4(w[r], next_bytes(w[r + 1], nx[r + 1]), sd);
  }
  acc[kT1] += t1;
  acc[kT2] += t2;
  acc[kSh] += sh;
  acc[kSv] += sv;
  acc[kSd] += sd;
  if (top) {
    acc[kR0S] += udot4(w[0], 0x01010101u, 0u);
    acc[kR0Q] += udot4(w[0], w[0], 0u);
  }
  if (bottom) {
    acc[kRLS] += udot4(w[7], 0x01010101u, 0u);
    acc[kRLQ] += udot4(w[7], w[7], 0u);
  }
  if (left) {
    uint32_t s = 0, q = 0;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const uint32_t b = w[r] & 0xffu;
      s += b;
      q += b * b;
    }
    acc[kC0S] += s;
    acc[kC0Q] += q;
    if (top) {
      const uint32_t b = w[0] & 0xffu;
      acc[kTLS] += b;
      acc[kTLQ] += b * b;
    }
  }
  if (right) {
    uint32_t s = 0, q = 0;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const uint32_t b = w[r] >> 24;
      s += b;
      q += b * b;
    }
    acc[kCLS] += s;
    acc[kCLQ] += q;
    if (bottom) {
      const uint32_t b = w[7] >> 24;
      acc[kBRS] += b;
      acc[kBRQ] += b * b;
    }
  }
}

// Block entropy of the lane's half block (lanes 2k, 2k + 1 share block k of
// the band): counts in LDS, then the product of the counts of the lane's 32
// samples' values.  sum_i log2(c_i) over the block is log2 of the two lanes'
// products (each count <= 64, so the product is at most 2^384: no overflow in
// FP64, relative error below 64 * 2^-53).
__device__ __forceinline__ double band_block_count_product(const uint32_t (&w)[9], uint32_t *cnt, int lane) {
  uint32_t *blk = cnt + (lane >> 1) * 64;
  // zero the wave's 32 x 64 counter words together: each store instruction
  // covers 1 KB of consecutive words (per-block 16-byte stores at a 128-byte
  // lane stride would all fall into the same few LDS banks)
  uint4 *z = reinterpret_cast<uint4 *>(cnt);
#pragma unroll
  for (int i = 0; i < 8; ++i) z[64 * i + lane] = make_uint4(0, 0, 0, 0);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  // one row at a time (sched_barrier): all 32 accesses in flight at once
  // would hold twice the registers for no gain
  // counter of value v: byte v of the block's 256-byte array
  uint8_t *bytes_w = reinterpret_cast<uint8_t *>(blk);
#pragma unroll
  for (int r = 0; r < 8; ++r) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint32_t v = (w[r] >> (8 * i)) & 0xffu;
      atomicAdd(reinterpret_cast<uint32_t *>(bytes_w + (v & 0xfcu)), 1u << ((v & 3u) << 3));
    }
    __builtin_amdgcn_sched_barrier(0);
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const uint8_t *bytes = reinterpret_cast<const uint8_t *>(blk);
  // products of four counts are exact integers (<= 2^24): multiply those in
  // 32-bit integers, then the eight partial products in FP64
  double p = 1.0;
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    uint32_t q = 1u;
#pragma unroll
    for (int i = 0; i < 4; ++i) q *= bytes[(w[r] >> (8 * i)) & 0xffu];
    p *= (double)q;
    __builtin_amdgcn_sched_barrier(0);
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  return p;
}

struct BandArgs {
  StatsGeom g;
  const uint8_t *x;
  const uint8_t *y;
  Partial *partials;  // kBandGrid slots
  float *block_entropy;  // optional: nb values for x, then nb for y
};

// Loads the lane's words of rows r0 .. r0 + 8 (row 8 is the next band's first
// row, zero past the plane) and the next lane's first bytes.
__device__ __forceinline__ void band_load(const uint8_t *img, const StatsGeom &g, uint32_t plane, uint32_t by,
                                          uint32_t wc, bool valid, int lane, uint32_t (&w)[9], uint32_t (&nx)[9]) {
  const uint8_t *base = img + (size_t)plane * g.H * g.W + (size_t)by * 8u * g.W;
  const bool has_below = by + 1u < g.By;
#pragma unroll
  for (int r = 0; r < 9; ++r) {
    const bool ok = valid && (r < 8 || has_below);
    w[r] = ok ? *reinterpret_cast<const uint32_t *>(base + (size_t)r * g.W + 4u * wc) : 0u;
  }
  // next word: from the next lane, or (last lane of the band) from memory
  const bool need_mem = lane == 63 && valid && wc + 1u < g.wpr;
#pragma unroll
  for (int r = 0; r < 9; ++r) {
    uint32_t v = __shfl_down(w[r], 1, 64);
    if (lane == 63) v = 0u;
    if (need_mem && (r < 8 || has_below)) v = *reinterpret_cast<const uint32_t *>(base + (size_t)r * g.W + 4u * wc + 4u);
    nx[r] = v;
  }
}

__global__ __launch_bounds__(kBandThreads) void stats_band_kernel(BandArgs a) {
  __shared__ __attribute__((aligned(16))) uint32_t s_cnt[kBandWaves][32 * 64];
  __shared__ Partial s_part[kBandWaves];
  const int lane = threadIdx.x & 63;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const StatsGeom &g = a.g;
  uint32_t acc[kIntMoments];
#pragma unroll
  for (int i = 0; i < kIntMoments; ++i) acc[i] = 0;
  if (lane == 0)
    for (int i = 0; i < kIntMoments; ++i) s_part[wave].m[i] = 0;
  // lane sums into the wave's 64-bit record, one sum at a time: interleaving
  // all of them holds every partial in registers at once, which is what would
  // set this kernel's register count
  auto flush = [&]() __attribute__((always_inline)) {
#pragma unroll
    for (int i = 0; i < kIntMoments; ++i) {
      const uint64_t v = wave_sum((uint64_t)acc[i]);
      if (lane == 0) s_part[wave].m[i] += v;
      acc[i] = 0;
      __builtin_amdgcn_sched_barrier(0);
    }
  };
  double esum[2] = {0.0, 0.0}, esq[2] = {0.0, 0.0};
  double emin[2] = {1e300, 1e300}, emax[2] = {-1e300, -1e300};
  const uint64_t nb = (uint64_t)g.C * g.By * g.Bx;
  uint32_t since_flush = 0;
  for (uint32_t band = blockIdx.x * kBandWaves + wave; band < g.nbands; band += gridDim.x * kBandWaves) {
    if (++since_flush > kFlushBands) {
      flush();
      since_flush = 1;
    }
    const uint32_t bx = band % g.nbx, rest = band / g.nbx;
    const uint32_t by = rest % g.By, plane = rest / g.By;
    const uint32_t wc = bx * 64u + (uint32_t)lane;
    const bool valid = wc < g.wpr;
    const bool top = by == 0, bottom = by + 1u == g.By, left = wc == 0, right = wc + 1u == g.wpr;
    const uint64_t blk = ((uint64_t)plane * g.By + by) * g.Bx + bx * 32u + (uint32_t)(lane >> 1);
    // X first; its eight row words stay for the X-Y terms while Y is processed
    uint32_t wx[8];
#pragma unroll
    for (int im = 0; im < 2; ++im) {
      uint32_t w[9], nx[9];
      band_load(im == 0 ? a.x : a.y, g, plane, by, wc, valid, lane, w, nx);
      if (valid) band_image_moments(w, nx, top, bottom, left, right, acc + im * kImgMoments);
      if (im == 0) {
#pragma unroll
        for (int r = 0; r < 8; ++r) wx[r] = w[r];
      } else if (valid) {
        uint32_t xy = 0, bits = 0;
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          xy = udot4(wx[r], w[r], xy);
          bits += (uint32_t)__builtin_popcount(wx[r] ^ w[r]);
        }
        acc[kCrossXY] += xy;
        acc[kBitsDiff] += bits;
      }
      // block entropy (every lane takes part in the LDS steps)
      double pr = band_block_count_product(w, s_cnt[wave], lane);
      pr *= __shfl_xor(pr, 1, 64);
      const double h = 6.0 - log2(pr) * (1.0 / 64.0);
      if (valid && (lane & 1) == 0) {
        esum[im] += h;
        esq[im] += h * h;
        emin[im] = fmin(emin[im], h);
        emax[im] = fmax(emax[im], h);
        if (a.block_entropy) a.block_entropy[(size_t)im * nb + blk] = (float)h;
      }
    }
  }
  // wave, then workgroup reduction into this workgroup's partial slot
  flush();
  double fl[kFltMoments];
#pragma unroll
  for (int im = 0; im < 2; ++im) {
    fl[4 * im + 0] = wave_sum(esum[im]);
    fl[4 * im + 1] = wave_sum(esq[im]);
    double mn = emin[im], mx = emax[im];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      mn = fmin(mn, __shfl_xor(mn, o, 64));
      mx = fmax(mx, __shfl_xor(mx, o, 64));
    }
    fl[4 * im + 2] = mn;
    fl[4 * im + 3] = mx;
  }
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < kFltMoments; ++i) s_part[wave].f[i] = fl[i];
  }
  __syncthreads();
  if (threadIdx.x < kIntMoments) {
    uint64_t v = 0;
    for (int w = 0; w < kBandWaves; ++w) v += s_part[w].m[threadIdx.x];
    a.partials[blockIdx.x].m[threadIdx.x] = v;
  } else if (threadIdx.x >= 64 && threadIdx.x < 64 + kFltMoments) {
    const int i = threadIdx.x - 64;
    double v = s_part[0].f[i];
    for (int w = 1; w < kBandWaves; ++w) {
      const double o = s_part[w].f[i];
      v = (i & 3) == 2 ? fmin(v, o) : (i & 3) == 3 ? fmax(v, o) : v + o;
    }
    a.partials[blockIdx.x].f[i] = v;
  }
}

// ---------------------------------------------------------------------------
__global__ void stats_clear_kernel(uint32_t *p, uint32_t n) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0u;
}

struct JointArgs {
  const uint4 *x;
  const uint4 *y;
  uint64_t nvec;       // samples / 16
  uint64_t per_chunk;  // vectors per workgroup
  uint32_t *hist;      // 65536 bins, bin = 256 x + y
};

__global__ __launch_bounds__(kJointThreads) void stats_joint_kernel(JointArgs a) {
  __shared__ uint32_t s_bins[kHalfBins];
  const uint32_t half = blockIdx.y;
  for (uint32_t i = threadIdx.x; i < kHalfBins; i += kJointThreads) s_bins[i] = 0u;
  __syncthreads();
  const uint64_t v0 = (uint64_t)blockIdx.x * a.per_chunk;
  const uint64_t v1 = min(a.nvec, v0 + a.per_chunk);
  for (uint64_t v = v0 + threadIdx.x; v < v1; v += kJointThreads) {
    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
    const u32x4 xv = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(&a.x[v]));
    const u32x4 yv = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(&a.y[v]));
    const uint32_t xw[4] = {xv[0], xv[1], xv[2], xv[3]}, yw[4] = {yv[0], yv[1], yv[2], yv[3]};
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const uint32_t xb = (xw[k] >> (8 * i)) & 0xffu, yb = (yw[k] >> (8 * i)) & 0xffu;
        if ((xb >> 7) == half) atomicAdd(&s_bins[((xb & 127u) << 8) | yb], 1u);
      }
  }
  __syncthreads();
  uint32_t *dst = a.hist + half * kHalfBins;
  for (uint32_t i = threadIdx.x; i < kHalfBins; i += kJointThreads) {
    const uint32_t c = s_bins[i];
    if (c) atomicAdd(&dst[i], c);
  }
}

// ---------------------------------------------------------------------------
// Reductions after the counting kernels, in the workspace (Reduced):
//  * rows kernel, one workgroup per joint-histogram row j (x = j): the row
//    sum (hist_x[j]), sum c log2 c over the row, and the column sums
//    (hist_y) by 64-bit integer atomics; workgroups j < kIntMoments +
//    kFltMoments also reduce one partial moment over the band workgroups.
//  * finalize, one workgroup: everything else, from 256-entry arrays.
// All floating sums use fixed trees, so the results do not depend on timing.
struct Reduced {
  uint64_t hx[256];
  uint64_t hy[256];
  double rowlog[256];
  uint64_t m[kIntMoments];
  double f[kFltMoments];
};

struct FinArgs {
  StatsGeom g;
  const Partial *partials;
  uint32_t nparts;
  const uint32_t *hist;
  Reduced *red;
  sf_security_stats *out;
};

typedef unsigned __int128 u128;
typedef __int128 i128;

// Pearson's r from exact moments; numerator and both variance factors as
// 128-bit integers.
__device__ double pearson(uint64_t n, uint64_t sx, uint64_t sy, uint64_t sxx, uint64_t syy, uint64_t sxy) {
  const i128 num = (i128)((u128)n * sxy) - (i128)((u128)sx * sy);
  const i128 dx = (i128)((u128)n * sxx) - (i128)((u128)sx * sx);
  const i128 dy = (i128)((u128)n * syy) - (i128)((u128)sy * sy);
  if (dx <= 0 || dy <= 0) return 0.0;
  return (double)num / sqrt((double)dx * (double)dy);
}

template <class T, class Op>
__device__ T block_reduce(T v, T *sh, Op op) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int s = kFinThreads / 2; s > 0; s >>= 1) {
    if (t < s) sh[t] = op(sh[t], sh[t + s]);
    __syncthreads();
  }
  const T r = sh[0];
  __syncthreads();
  return r;
}

__device__ double block_sum(double v, double *sh) {
  return block_reduce(v, sh, [](double a, double b) { return a + b; });
}

__device__ double clog2c(uint64_t c) { return c ? (double)c * log2((double)c) : 0.0; }

__global__ __launch_bounds__(kFinThreads) void stats_rows_kernel(FinArgs a) {
  __shared__ double s_d[kFinThreads];
  __shared__ uint64_t s_u[kFinThreads];
  const int t = threadIdx.x;
  const uint32_t j = blockIdx.x;
  const uint32_t c = a.hist[j * 256u + t];
  atomicAdd(reinterpret_cast<unsigned long long *>(&a.red->hy[t]), (unsigned long long)c);
  const uint64_t rs = block_reduce<uint64_t>(c, s_u, [](uint64_t x, uint64_t y) { return x + y; });
  const double rl = block_sum(clog2c(c), s_d);
  if (t == 0) {
    a.red->hx[j] = rs;
    a.red->rowlog[j] = rl;
  }
  // one partial moment per workgroup: a fixed split over the threads, then a tree
  if (j < (uint32_t)kIntMoments) {
    uint64_t v = 0;
    for (uint32_t p = t; p < a.nparts; p += kFinThreads) v += a.partials[p].m[j];
    v = block_reduce<uint64_t>(v, s_u, [](uint64_t x, uint64_t y) { return x + y; });
    if (t == 0) a.red->m[j] = v;
  } else if (j < (uint32_t)(kIntMoments + kFltMoments)) {
    const int i = (int)j - kIntMoments;
    const int kind = i & 3;  // 0, 1: sums; 2: min; 3: max
    double v = kind == 2 ? 1e300 : kind == 3 ? -1e300 : 0.0;
    for (uint32_t p = t; p < a.nparts; p += kFinThreads) {
      const double w = a.partials[p].f[i];
      v = kind == 2 ? fmin(v, w) : kind == 3 ? fmax(v, w) : v + w;
    }
    v = block_reduce<double>(v, s_d, [kind](double x, double y) {
      return kind == 2 ? fmin(x, y) : kind == 3 ? fmax(x, y) : x + y;
    });
    if (t == 0) a.red->f[i] = v;
  }
}

// Four sums over the block's threads in one fixed LDS tree (deterministic).
__device__ void block_sum4(double (&v)[4], double (*sh)[kFinThreads]) {
  const int t = threadIdx.x;
#pragma unroll
  for (int q = 0; q < 4; ++q) sh[q][t] = v[q];
  __syncthreads();
  for (int s = kFinThreads / 2; s > 0; s >>= 1) {
    if (t < s)
#pragma unroll
      for (int q = 0; q < 4; ++q) sh[q][t] += sh[q][t + s];
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) v[q] = sh[q][0];
}

// One thread per bin for the histogram sums; the scalar results are then
// spread over threads: 0 entropies, 0-5 one (image, direction) pair
// correlation each, 6 the image-pair figures, 7 the block-entropy summaries.
__global__ __launch_bounds__(kFinThreads) void stats_finalize_kernel(FinArgs a) {
  __shared__ uint64_t s_m[kIntMoments];
  __shared__ double s_f[kFltMoments];
  __shared__ double s_red[4][kFinThreads];
  const int t = threadIdx.x;
  const StatsGeom &g = a.g;
  sf_security_stats *o = a.out;
  const Reduced *rd = a.red;
  if (t < kIntMoments) s_m[t] = rd->m[t];
  else if (t >= 64 && t < 64 + kFltMoments) s_f[t - 64] = rd->f[t - 64];
  const uint64_t hx = rd->hx[t], hy = rd->hy[t];
  o->hist_x[t] = hx;
  o->hist_y[t] = hy;
  const uint64_t N = (uint64_t)g.C * g.H * g.W;
  const double dN = (double)N;
  const double e = dN / 256.0;
  double v[4] = {((double)hy - e) * ((double)hy - e) / e, clog2c(hx), clog2c(hy), rd->rowlog[t]};
  block_sum4(v, s_red);  // its barriers also publish s_m and s_f
  if (t == 0) {
    o->samples = N;
    const double lN = log2(dN);
    const double Hx = lN - v[1] / dN, Hy = lN - v[2] / dN, Hxy = lN - v[3] / dN;
    o->chi2_y = v[0];
    o->entropy_x = Hx;
    o->entropy_y = Hy;
    o->joint_entropy = Hxy;
    o->mutual_information = Hx + Hy - Hxy;
    o->nmi = Hx * Hy > 0.0 ? (Hx + Hy - Hxy) / sqrt(Hx * Hy) : 0.0;
  }
  if (t < 6) {
    // directional pair moments from whole-plane and border sums; h: x drops
    // the last column, y the first; v: rows; d: both
    const int im = t / 3, d = t - 3 * (t / 3);
    const uint64_t C = g.C, H = g.H, W = g.W;
    const uint64_t *m = s_m + im * kImgMoments;
    uint64_t n, sx, sy, qx, qy, pr;
    if (d == 0) {
      n = C * H * (W - 1);
      sx = m[kT1] - m[kCLS];
      sy = m[kT1] - m[kC0S];
      qx = m[kT2] - m[kCLQ];
      qy = m[kT2] - m[kC0Q];
      pr = m[kSh];
    } else if (d == 1) {
      n = C * (H - 1) * W;
      sx = m[kT1] - m[kRLS];
      sy = m[kT1] - m[kR0S];
      qx = m[kT2] - m[kRLQ];
      qy = m[kT2] - m[kR0Q];
      pr = m[kSv];
    } else {
      n = C * (H - 1) * (W - 1);
      sx = m[kT1] - m[kRLS] - m[kCLS] + m[kBRS];
      sy = m[kT1] - m[kR0S] - m[kC0S] + m[kTLS];
      qx = m[kT2] - m[kRLQ] - m[kCLQ] + m[kBRQ];
      qy = m[kT2] - m[kR0Q] - m[kC0Q] + m[kTLQ];
      pr = m[kSd];
    }
    uint64_t *pm = (im == 0 ? o->pair_x : o->pair_y)[d];
    pm[0] = n;
    pm[1] = sx;
    pm[2] = sy;
    pm[3] = qx;
    pm[4] = qy;
    pm[5] = pr;
    (im == 0 ? o->corr_x : o->corr_y)[d] = pearson(n, sx, sy, qx, qy, pr);
  } else if (t == 6) {
    const uint64_t sx = s_m[kT1], sy = s_m[kImgMoments + kT1];
    const uint64_t sxx = s_m[kT2], syy = s_m[kImgMoments + kT2], sxy = s_m[kCrossXY];
    o->cross[0] = N;
    o->cross[1] = sx;
    o->cross[2] = sy;
    o->cross[3] = sxx;
    o->cross[4] = syy;
    o->cross[5] = sxy;
    o->bits_differing = s_m[kBitsDiff];
    o->corr2 = pearson(N, sx, sy, sxx, syy, sxy);
    o->dif = 100.0 * (double)s_m[kBitsDiff] / (8.0 * dN);
    const uint64_t sse = sxx + syy - 2u * sxy;  // sum (x - y)^2, exact
    o->psnr = sse == 0 ? __builtin_huge_val() : 10.0 * log10(65025.0 * dN / (double)sse);
  } else if (t == 7) {
    const double nbk = (double)((uint64_t)g.C * g.By * g.Bx);
    for (int im = 0; im < 2; ++im) {
      double *be = im == 0 ? o->block_entropy_x : o->block_entropy_y;
      const double mean = s_f[4 * im] / nbk;
      const double var = s_f[4 * im + 1] / nbk - mean * mean;
      be[0] = mean;
      be[1] = var > 0.0 ? sqrt(var) : 0.0;
      be[2] = s_f[4 * im + 2];
      be[3] = s_f[4 * im + 3];
    }
  }
}

StatsGeom stats_geom(uint32_t H, uint32_t W, uint32_t C) {
  StatsGeom g;
  g.H = H;
  g.W = W;
  g.C = C;
  g.By = H / 8;
  g.Bx = W / 8;
  g.wpr = W / 4;
  g.nbx = (g.wpr + 63) / 64;
  g.nbands = C * g.By * g.nbx;
  return g;
}

}  // namespace

constexpr size_t kHistBytes = 65536 * sizeof(uint32_t);
constexpr size_t kPartBytes = kBandGrid * sizeof(Partial);
static_assert(kHistBytes % 16 == 0 && kPartBytes % 16 == 0, "workspace parts stay 16-byte aligned");

size_t stats_workspace_bytes() { return kHistBytes + kPartBytes + sizeof(Reduced); }

int launch_security_stats(const DeviceState &ds, const uint8_t *x, const uint8_t *y, uint32_t H, uint32_t W,
                          uint32_t C, void *ws, sf_security_stats *out, float *block_entropy, hipStream_t stream) {
  const StatsGeom g = stats_geom(H, W, C);
  uint32_t *hist = static_cast<uint32_t *>(ws);
  Partial *parts = reinterpret_cast<Partial *>(static_cast<uint8_t *>(ws) + kHistBytes);
  Reduced *red = reinterpret_cast<Reduced *>(static_cast<uint8_t *>(ws) + kHistBytes + kPartBytes);
  // the histogram and the column sums start at zero (a fill kernel, not a
  // memset, so the sequence can be captured in a graph)
  hipLaunchKernelGGL(stats_clear_kernel, dim3(64), dim3(256), 0, stream, hist, 65536u);
  hipLaunchKernelGGL(stats_clear_kernel, dim3(1), dim3(256), 0, stream, reinterpret_cast<uint32_t *>(red->hy),
                     (uint32_t)(sizeof(red->hy) / 4));
  BandArgs b{g, x, y, parts, block_entropy};
  // one generation of resident workgroups (more would leave a partly empty
  // last generation), at most kBandGrid partial slots
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)&stats_band_kernel, kBandThreads, 0) !=
          hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  const uint32_t need = (g.nbands + kBandWaves - 1) / kBandWaves;
  uint32_t grid = std::min<uint32_t>((uint32_t)ds.num_cu * (uint32_t)per_cu, (uint32_t)kBandGrid);
  grid = std::min(grid, need);
  // unused partial slots are read by the finalize kernel: it takes only `grid`
  hipLaunchKernelGGL(stats_band_kernel, dim3(grid), dim3(kBandThreads), 0, stream, b);
  JointArgs j;
  j.x = reinterpret_cast<const uint4 *>(x);
  j.y = reinterpret_cast<const uint4 *>(y);
  j.nvec = (uint64_t)C * H * W / 16u;
  // 128 KB of LDS: one workgroup per CU; two per chunk (the halves), so
  // num_cu / 2 chunks fill the chip in one generation
  const uint64_t chunks = std::max<uint64_t>(1, std::min<uint64_t>((uint64_t)ds.num_cu / 2u, j.nvec / 16384u));
  j.per_chunk = (j.nvec + chunks - 1) / chunks;
  j.hist = hist;
  hipLaunchKernelGGL(stats_joint_kernel, dim3((uint32_t)chunks, 2), dim3(kJointThreads), 0, stream, j);
  FinArgs f{g, parts, grid, hist, red, out};
  hipLaunchKernelGGL(stats_rows_kernel, dim3(256), dim3(kFinThreads), 0, stream, f);
  hipLaunchKernelGGL(stats_finalize_kernel, dim3(1), dim3(kFinThreads), 0, stream, f);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SF_OK : hip_fail(e, "security statistics launch");
}

}  // namespace sf
