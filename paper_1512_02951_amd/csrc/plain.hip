// Plain (FP32) form of the first level of protection: one wavefront per tile
// of 64 consecutive 8x8 blocks, one block per lane.  The per-tile bodies are
// in plain_tile.h (shared with the batched persistent kernel); this file holds
// the single-image kernels and their launchers.  Each call is one kernel
// launch: exceptions live in per-tile slots, so there is no counter to clear
// and no separate pass to apply them.
#include "plain_tile.h"

namespace sf {
namespace {

// Workgroups of 1 to 8 wavefronts (the launch shape; 2 is the default).
constexpr int kMaxWaves = 8;
constexpr int kMaxThreads = 64 * kMaxWaves;

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

// Each wave walks tiles t, t + stride, ... (kLoop, the resident grids), or
// takes the one tile t (one tile per wave: no loop and no prefetch of a next
// tile, whose 16 pixel words would otherwise stay live through the tile).
// kQ2Mfma: the private AC integers come from int8 matrix products (at most
// 16 private AC coefficients); each wave then owns kQ2StageBytes of LDS
// after its private-byte staging area.
template <class MP, bool kQ2Mfma, bool kLoop>
__global__ __launch_bounds__(kMaxThreads, SF_FRAG_WAVES_PER_EU) void frag_fp32_kernel(FragKernelArgs a) {
  __shared__ AesLds s_aes;
  __shared__ Q2Operands s_q2[kQ2Mfma ? 64 : 1];  // B operand per lane (same for every wave)
  extern __shared__ __attribute__((aligned(16))) uint8_t s_dyn[];
  const int lane = threadIdx.x & 63;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint32_t nw = blockDim.x >> 6;
  if (a.aes.enabled) aes_load_tables(s_aes, a.aes_t0, a.aes.key, threadIdx.x, blockDim.x);
  if constexpr (kQ2Mfma)
    if (threadIdx.x < 64) s_q2[lane] = q2_operands(a.o.q2, private_ac<MP>(a.g.mask, lane & 15), lane);
  __syncthreads();
  constexpr uint32_t kStage = kQ2Mfma ? kQ2StageBytes : 0u;
  uint8_t *lp = s_dyn + wave * (a.lds_priv_bytes + kStage);
  uint8_t *q2stage = lp + a.lds_priv_bytes;
  const Q2Operands *Q = &s_q2[kQ2Mfma ? lane : 0];
  const uint32_t stride = gridDim.x * nw;
  uint32_t t = blockIdx.x * nw + wave;
  if (t >= a.g.ntiles) return;
  if constexpr (!kLoop) {
    const TileLane L = tile_lane(a.g, t, lane);
    uint32_t xs[16];
    load_block(a.g, L, xs);
    if constexpr (kQ2Mfma)
      frag_tile<MP, true>(a.g, a.o, t, L, xs, lane, lp, s_aes, a.aes.enabled, a.aes.ctr_hi, a.aes.ctr_lo, a.K,
                          q2stage, Q);
    else
      frag_tile<MP, false>(a.g, a.o, t, L, xs, lane, lp, s_aes, a.aes.enabled, a.aes.ctr_hi, a.aes.ctr_lo, a.K);
    return;
  }
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
__global__ __launch_bounds__(kMaxThreads, SF_DEFRAG_WAVES_PER_EU) void defrag_fp32_kernel(DefragKernelArgs a) {
  __shared__ AesLds s_aes;
  extern __shared__ __attribute__((aligned(16))) uint8_t s_dyn[];
  const int lane = threadIdx.x & 63;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint32_t nw = blockDim.x >> 6;
  if (a.aes.enabled) aes_load_tables(s_aes, a.aes_t0, a.aes.key, threadIdx.x, blockDim.x);
  __syncthreads();
  uint8_t *lp = s_dyn + wave * a.lds_priv_bytes;
  const uint32_t stride = gridDim.x * nw;
  for (uint32_t t = blockIdx.x * nw + wave; t < a.g.ntiles; t += stride)
    defrag_tile<MP>(a.g, a.in, t, tile_lane(a.g, t, lane), lane, lp, s_aes, a.aes.enabled, a.aes.ctr_hi,
                    a.aes.ctr_lo, a.K);
}

uint32_t lds_priv_bytes(const Geom &g) { return (2u * g.npriv * 64u + 15u) & ~15u; }

// resident = 1: as many workgroups as the device holds at once, each wave
// looping over tiles; resident = 0: one tile per wave, the hardware
// dispatcher refilling SIMDs as waves finish.
// Beyond 2^31 - 1 workgroups the grid is capped at that (the kernels loop).
int grid_for(const DeviceState &ds, const void *kernel, const Shape &sh, size_t lds, uint32_t ntiles) {
  uint64_t need = ((uint64_t)ntiles + sh.waves - 1) / sh.waves;
  if (sh.resident) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 64 * (int)sh.waves, lds) != hipSuccess ||
        per_cu < 1)
      per_cu = 1;
    const uint64_t cap = (uint64_t)ds.num_cu * (uint64_t)per_cu;
    need = need < cap ? need : cap;
  }
  return (int)(need < 0x7fffffffu ? need : 0x7fffffffu);
}

bool q2_on_mfma(const Geom &g) { return __builtin_popcountll(g.mask & ~1ull) <= kQ2MfmaMaxAc; }

template <class MP, bool kQ2Mfma>
int launch_frag_mp(const DeviceState &ds, const FragKernelArgs &a, const Shape &sh, hipStream_t stream) {
  const size_t lds = (size_t)sh.waves * (a.lds_priv_bytes + (kQ2Mfma ? kQ2StageBytes : 0u));
  void (*kern)(FragKernelArgs) = sh.resident ? frag_fp32_kernel<MP, kQ2Mfma, true> : frag_fp32_kernel<MP, kQ2Mfma, false>;
  const int grid = grid_for(ds, (const void *)kern, sh, lds, a.g.ntiles);
  hipLaunchKernelGGL(kern, dim3(grid), dim3(64 * sh.waves), lds, stream, a);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SF_OK : hip_fail(e, "frag kernel launch");
}

template <class MP>
int launch_defrag_mp(const DeviceState &ds, const DefragKernelArgs &a, const Shape &sh, hipStream_t stream) {
  const size_t lds = (size_t)sh.waves * a.lds_priv_bytes;
  const int grid = grid_for(ds, (const void *)&defrag_fp32_kernel<MP>, sh, lds, a.g.ntiles);
  hipLaunchKernelGGL(defrag_fp32_kernel<MP>, dim3(grid), dim3(64 * sh.waves), lds, stream, a);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SF_OK : hip_fail(e, "defrag kernel launch");
}

// The resolved shape, or SF_ENOTSUP if its LDS does not fit a workgroup.
int plain_shape(const DeviceState &ds, const Geom &g, int which, const Shape &in, Shape *out) {
  *out = in;
  if (!out->waves) out->waves = plain_default_waves(g, which);
  if (out->waves > (uint32_t)kMaxWaves || plain_lds_bytes(g, which, out->waves) > ds.max_lds_per_block)
    return fail(SF_ENOTSUP, "launch shape: the workgroup's LDS does not fit on this device");
  return SF_OK;
}

}  // namespace

size_t plain_lds_bytes(const Geom &g, int which, uint32_t waves) {
  const size_t priv = lds_priv_bytes(g);
  if (which == 1) return sizeof(AesLds) + waves * priv;
  const bool mf = q2_on_mfma(g);
  return sizeof(AesLds) + (mf ? 64u : 1u) * sizeof(Q2Operands) + waves * (priv + (mf ? kQ2StageBytes : 0u));
}

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
                     const sf_exceptions *exc, const AesArgs &aes, uint32_t *status, const Shape &shape,
                     hipStream_t stream) {
  Shape sh;
  if (int rc = plain_shape(ds, g, 0, shape, &sh)) return rc;
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
    case (1ull << 2) - 1: return launch_frag_mp<MaskPrefix<2>, true>(ds, a, sh, stream);
    case (1ull << 3) - 1: return launch_frag_mp<MaskPrefix<3>, true>(ds, a, sh, stream);
    case (1ull << 6) - 1: return launch_frag_mp<MaskPrefix<6>, true>(ds, a, sh, stream);
    case (1ull << 10) - 1: return launch_frag_mp<MaskPrefix<10>, true>(ds, a, sh, stream);
    default:
      if (q2_on_mfma(g)) return launch_frag_mp<MaskRuntime, true>(ds, a, sh, stream);
      return launch_frag_mp<MaskRuntime, false>(ds, a, sh, stream);
  }
}

int launch_defrag_fp32(const DeviceState &ds, const Geom &g, const float *pub, const uint8_t *priv,
                       const sf_exceptions *exc, const AesArgs &aes, uint8_t *pix, const Shape &shape,
                       hipStream_t stream) {
  Shape sh;
  if (int rc = plain_shape(ds, g, 1, shape, &sh)) return rc;
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
  switch (g.mask) {
    case (1ull << 2) - 1: return launch_defrag_mp<MaskPrefix<2>>(ds, a, sh, stream);
    case (1ull << 3) - 1: return launch_defrag_mp<MaskPrefix<3>>(ds, a, sh, stream);
    case (1ull << 6) - 1: return launch_defrag_mp<MaskPrefix<6>>(ds, a, sh, stream);
    case (1ull << 10) - 1: return launch_defrag_mp<MaskPrefix<10>>(ds, a, sh, stream);
    default: return launch_defrag_mp<MaskRuntime>(ds, a, sh, stream);
  }
}

}  // namespace sf
