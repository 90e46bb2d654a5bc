// Plain (FP32) form of the first level of protection: one wavefront per tile
// of 64 consecutive 8x8 blocks, one block per lane.  The per-tile bodies are
// in plain_tile.h (shared with the batched persistent kernel); this file holds
// the single-image kernels and their launchers.  Each call is one kernel
// launch: exceptions live in per-tile slots, so there is no counter to clear
// and no separate pass to apply them.
#include "plain_tile.h"

namespace sf {
namespace {

constexpr int kWaves = 2;  // 2 waves per workgroup measured best (1, 2, 4, 8 tried)
constexpr int kThreads = 64 * kWaves;

struct FragKernelArgs {
  TileGeom g;
  FragOut o;
  const uint32_t *aes_t0;
  AesArgs aes;
  DctK K;
  uint32_t lds_priv_bytes;
};

struct DefragKernelArgs {
  TileGeom g;
  DefragIn in;
  const uint32_t *aes_t0;
  AesArgs aes;
  DctK K;
  uint32_t lds_priv_bytes;
};

// Tuning knobs (compile-time): minimum waves per SIMD requested from the
// register allocator, and whether frag loads the next tile's pixels before
// working on the current one.
#ifndef SF_FRAG_WAVES_PER_EU
#define SF_FRAG_WAVES_PER_EU 3
#endif
#ifndef SF_DEFRAG_WAVES_PER_EU
#define SF_DEFRAG_WAVES_PER_EU 3
#endif
#ifndef SF_FRAG_PREFETCH
#define SF_FRAG_PREFETCH 0
#endif

// Each wave walks tiles t, t + stride, ...
// kQ2Mfma: the private AC integers come from int8 matrix products (at most
// 16 private AC coefficients); each wave then owns kQ2StageBytes of LDS
// after its private-byte staging area.
template <class MP, bool kQ2Mfma>
__global__ __launch_bounds__(kThreads, SF_FRAG_WAVES_PER_EU) void frag_fp32_kernel(FragKernelArgs a) {
  __shared__ AesLds s_aes;
  __shared__ Q2Operands s_q2[kQ2Mfma ? 64 : 1];  // B operand per lane (same for every wave)
  extern __shared__ __attribute__((aligned(16))) uint8_t s_dyn[];
  const int lane = threadIdx.x & 63;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (a.aes.enabled) aes_load_tables(s_aes, a.aes_t0, a.aes.key, threadIdx.x, kThreads);
  if constexpr (kQ2Mfma)
    if (threadIdx.x < 64) s_q2[lane] = q2_operands(a.o.q2, private_ac<MP>(a.g.mask, lane & 15), lane);
  __syncthreads();
  constexpr uint32_t kStage = kQ2Mfma ? kQ2StageBytes : 0u;
  uint8_t *lp = s_dyn + wave * (a.lds_priv_bytes + kStage);
  uint8_t *q2stage = lp + a.lds_priv_bytes;
  const Q2Operands *Q = &s_q2[kQ2Mfma ? lane : 0];
  const uint32_t stride = gridDim.x * kWaves;
  uint32_t t = blockIdx.x * kWaves + wave;
  if (t >= a.g.ntiles) return;
#if SF_FRAG_PREFETCH
  TileLane L = tile_lane(a.g, t, lane);
  uint32_t xs[16];
  load_block(a.g, L, xs);
  for (;;) {
    const uint32_t tn = t + stride;
    const bool more = tn < a.g.ntiles;
    TileLane Ln = L;
    uint32_t xn[16];
    if (more) {
      Ln = tile_lane(a.g, tn, lane);
      load_block(a.g, Ln, xn);
    }
    frag_tile<MP, kQ2Mfma>(a.g, a.o, t, L, xs, lane, lp, s_aes, a.aes.enabled, a.aes.ctr_hi, a.aes.ctr_lo, a.K,
                           q2stage, Q);
    if (!more) break;
    t = tn;
    L = Ln;
#pragma unroll
    for (int w = 0; w < 16; ++w) xs[w] = xn[w];
  }
#else
  if constexpr (kQ2Mfma) {
    // the next tile's pixels are loaded from inside frag_tile, once the
    // current ones have been consumed
    TileLane L = tile_lane(a.g, t, lane);
    uint32_t xs[16];
    load_block(a.g, L, xs);
    for (;;) {
      const uint32_t tn = t + stride;
      const bool more = tn < a.g.ntiles;
      const TileLane Ln = more ? tile_lane(a.g, tn, lane) : L;
      frag_tile<MP, true>(a.g, a.o, t, L, xs, lane, lp, s_aes, a.aes.enabled, a.aes.ctr_hi, a.aes.ctr_lo, a.K,
                          q2stage, Q, [&]() {
                            if (more) load_block(a.g, Ln, xs);
                          });
      if (!more) break;
      t = tn;
      L = Ln;
    }
  } else {
    for (; t < a.g.ntiles; t += stride) {
      const TileLane L = tile_lane(a.g, t, lane);
      uint32_t xs[16];
      load_block(a.g, L, xs);
      frag_tile<MP, false>(a.g, a.o, t, L, xs, lane, lp, s_aes, a.aes.enabled, a.aes.ctr_hi, a.aes.ctr_lo, a.K);
    }
  }
#endif
}

template <class MP>
__global__ __launch_bounds__(kThreads, SF_DEFRAG_WAVES_PER_EU) void defrag_fp32_kernel(DefragKernelArgs a) {
  __shared__ AesLds s_aes;
  extern __shared__ __attribute__((aligned(16))) uint8_t s_dyn[];
  const int lane = threadIdx.x & 63;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (a.aes.enabled) aes_load_tables(s_aes, a.aes_t0, a.aes.key, threadIdx.x, kThreads);
  __syncthreads();
  uint8_t *lp = s_dyn + wave * a.lds_priv_bytes;
  const uint32_t stride = gridDim.x * kWaves;
  for (uint32_t t = blockIdx.x * kWaves + wave; t < a.g.ntiles; t += stride)
    defrag_tile<MP>(a.g, a.in, t, tile_lane(a.g, t, lane), lane, lp, s_aes, a.aes.enabled, a.aes.ctr_hi,
                    a.aes.ctr_lo, a.K);
}

uint32_t lds_priv_bytes(const Geom &g) { return (2u * g.npriv * 64u + 15u) & ~15u; }

// One tile per wave: the hardware dispatcher keeps every SIMD at its
// occupancy limit and refills it as waves finish, which measured faster than
// resident waves looping over tiles (the kernels still loop if the grid is
// ever capped).  Beyond 2^31 - 1 workgroups the grid is capped at that.
int grid_for(const DeviceState &, const void *, size_t, uint32_t ntiles) {
  const uint64_t need = ((uint64_t)ntiles + kWaves - 1) / kWaves;
  return (int)(need < 0x7fffffffu ? need : 0x7fffffffu);
}

template <class MP, bool kQ2Mfma>
int launch_frag_mp(const DeviceState &ds, const FragKernelArgs &a, hipStream_t stream) {
  const size_t lds = (size_t)kWaves * (a.lds_priv_bytes + (kQ2Mfma ? kQ2StageBytes : 0u));
  const int grid = grid_for(ds, (const void *)&frag_fp32_kernel<MP, kQ2Mfma>, lds, a.g.ntiles);
  hipLaunchKernelGGL((frag_fp32_kernel<MP, kQ2Mfma>), dim3(grid), dim3(kThreads), lds, stream, a);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SF_OK : hip_fail(e, "frag kernel launch");
}

template <class MP>
int launch_defrag_mp(const DeviceState &ds, const DefragKernelArgs &a, size_t lds, hipStream_t stream) {
  const int grid = grid_for(ds, (const void *)&defrag_fp32_kernel<MP>, lds, a.g.ntiles);
  hipLaunchKernelGGL(defrag_fp32_kernel<MP>, dim3(grid), dim3(kThreads), lds, stream, a);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SF_OK : hip_fail(e, "defrag kernel launch");
}

}  // namespace

ExcSlots exc_slots(const Geom &g, const sf_exceptions *exc) {
  ExcSlots s{};
  s.check = mask_needs_check(g.mask) ? 1u : 0u;
  if (!s.check) return s;
  const ExcLayout lay = exc_layout(g, exc->per_tile);
  uint8_t *base = (uint8_t *)exc->d_buf;
  s.count = (uint16_t *)base;
  s.pos = (uint16_t *)(base + lay.pos_offset);
  s.val = base + lay.val_offset;
  s.per_tile = exc->per_tile;
  return s;
}

int launch_frag_fp32(const DeviceState &ds, const Geom &g, const uint8_t *pix, float *pub, uint8_t *priv,
                     const sf_exceptions *exc, const AesArgs &aes, uint32_t *status, hipStream_t stream) {
  FragKernelArgs a;
  a.g = tile_geom(g, pix);
  a.o.pub = pub;
  a.o.priv = priv;
  a.o.exc = exc_slots(g, exc);
  a.o.status = status;
  a.o.q2 = ds.d_q2;
  a.o.cert_thr = cert_threshold();
  a.aes_t0 = ds.d_aes_t0;
  a.aes = aes;
  a.K = host_tables().dct;
  a.lds_priv_bytes = lds_priv_bytes(g);
  // compile-time selections for DC + k AC, k in {1, 2, 5, 9}; any other mask
  // at run time, on the matrix cores while at most 16 AC coefficients are private
  switch (g.mask) {
    case (1ull << 2) - 1: return launch_frag_mp<MaskPrefix<2>, true>(ds, a, stream);
    case (1ull << 3) - 1: return launch_frag_mp<MaskPrefix<3>, true>(ds, a, stream);
    case (1ull << 6) - 1: return launch_frag_mp<MaskPrefix<6>, true>(ds, a, stream);
    case (1ull << 10) - 1: return launch_frag_mp<MaskPrefix<10>, true>(ds, a, stream);
    default:
      if (__builtin_popcountll(g.mask & ~1ull) <= kQ2MfmaMaxAc) return launch_frag_mp<MaskRuntime, true>(ds, a, stream);
      return launch_frag_mp<MaskRuntime, false>(ds, a, stream);
  }
}

int launch_defrag_fp32(const DeviceState &ds, const Geom &g, const float *pub, const uint8_t *priv,
                       const sf_exceptions *exc, const AesArgs &aes, uint8_t *pix, hipStream_t stream) {
  DefragKernelArgs a;
  a.g = tile_geom(g, nullptr);
  a.in.pix_out = pix;
  a.in.pub = pub;
  a.in.priv = priv;
  a.in.exc = exc_slots(g, exc);
  a.aes_t0 = ds.d_aes_t0;
  a.aes = aes;
  a.K = host_tables().dct;
  a.lds_priv_bytes = lds_priv_bytes(g);
  const size_t lds = (size_t)kWaves * a.lds_priv_bytes;
  switch (g.mask) {
    case (1ull << 2) - 1: return launch_defrag_mp<MaskPrefix<2>>(ds, a, lds, stream);
    case (1ull << 3) - 1: return launch_defrag_mp<MaskPrefix<3>>(ds, a, lds, stream);
    case (1ull << 6) - 1: return launch_defrag_mp<MaskPrefix<6>>(ds, a, lds, stream);
    case (1ull << 10) - 1: return launch_defrag_mp<MaskPrefix<10>>(ds, a, lds, stream);
    default: return launch_defrag_mp<MaskRuntime>(ds, a, lds, stream);
  }
}

}  // namespace sf
