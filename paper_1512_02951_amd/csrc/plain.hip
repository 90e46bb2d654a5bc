// Plain (FP32) form of the first level of protection: one wavefront per tile
// of 64 consecutive 8x8 blocks, one block per lane.  The per-tile bodies are
// in plain_tile.h (shared with the batched persistent kernel); this file holds
// the single-image kernels and their launchers.
#include "plain_tile.h"

namespace sf {
namespace {

constexpr int kWaves = 4;
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

__global__ void reset_count_kernel(uint32_t *count) { *count = 0u; }

template <class MP>
__global__ __launch_bounds__(kThreads) void frag_fp32_kernel(FragKernelArgs a) {
  __shared__ AesLds s_aes;
  extern __shared__ __attribute__((aligned(16))) uint8_t s_dyn[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (a.aes.enabled) aes_load_tables(s_aes, a.aes_t0, a.aes.key, threadIdx.x, kThreads);
  __syncthreads();
  uint8_t *lp = s_dyn + wave * a.lds_priv_bytes;
  const uint32_t nwaves = gridDim.x * kWaves;
  for (uint32_t t = blockIdx.x * kWaves + wave; t < a.g.ntiles; t += nwaves)
    frag_tile<MP>(a.g, a.o, t, lane, lp, s_aes, a.aes.enabled, a.aes.ctr_hi, a.aes.ctr_lo, 0u, a.K);
}

template <class MP>
__global__ __launch_bounds__(kThreads) void defrag_fp32_kernel(DefragKernelArgs a) {
  __shared__ AesLds s_aes;
  extern __shared__ __attribute__((aligned(16))) uint8_t s_dyn[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (a.aes.enabled) aes_load_tables(s_aes, a.aes_t0, a.aes.key, threadIdx.x, kThreads);
  __syncthreads();
  uint8_t *lp = s_dyn + wave * a.lds_priv_bytes;
  const uint32_t nwaves = gridDim.x * kWaves;
  for (uint32_t t = blockIdx.x * kWaves + wave; t < a.g.ntiles; t += nwaves)
    defrag_tile<MP>(a.g, a.in, t, lane, lp, s_aes, a.aes.enabled, a.aes.ctr_hi, a.aes.ctr_lo, 0u, a.K);
}

__global__ void apply_exceptions_kernel(const uint32_t *count, const uint32_t *index, const uint8_t *value,
                                        uint32_t cap, uint8_t *pix, uint32_t nsamples, uint32_t *status) {
  const uint32_t n0 = *count;
  const uint32_t n = n0 < cap ? n0 : cap;
  if (n0 > cap && status && blockIdx.x == 0 && threadIdx.x == 0) atomicOr(status, SF_STATUS_EXC_OVERFLOW);
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const uint32_t s = index[i];
    if (s < nsamples) pix[s] = value[i];
  }
}

uint32_t lds_priv_bytes(const Geom &g) { return (2u * g.npriv * 64u + 15u) & ~15u; }

int grid_for(const DeviceState &ds, const void *kernel, size_t lds, uint32_t ntiles) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kThreads, lds) != hipSuccess || per_cu < 1)
    per_cu = 1;
  const uint32_t need = (ntiles + kWaves - 1) / kWaves;
  const uint32_t cap = (uint32_t)ds.num_cu * (uint32_t)per_cu;
  return (int)(need < cap ? need : cap);
}

template <class MP>
int launch_frag_mp(const DeviceState &ds, const FragKernelArgs &a, size_t lds, hipStream_t stream) {
  const int grid = grid_for(ds, (const void *)&frag_fp32_kernel<MP>, lds, a.g.ntiles);
  hipLaunchKernelGGL(frag_fp32_kernel<MP>, dim3(grid), dim3(kThreads), lds, stream, a);
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

int launch_frag_fp32(const DeviceState &ds, const Geom &g, const uint8_t *pix, float *pub, uint8_t *priv,
                     const sf_exceptions &exc, const AesArgs &aes, uint32_t *status, hipStream_t stream) {
  FragKernelArgs a;
  a.g = tile_geom(g, pix);
  a.o.pub = pub;
  a.o.priv = priv;
  a.o.exc_count = exc.d_count;
  a.o.exc_index = exc.d_index;
  a.o.exc_value = exc.d_value;
  a.o.exc_cap = exc.capacity;
  a.o.status = status;
  a.o.q2 = ds.d_q2;
  a.aes_t0 = ds.d_aes_t0;
  a.aes = aes;
  a.K = host_tables().dct;
  a.lds_priv_bytes = lds_priv_bytes(g);
  const size_t lds = (size_t)kWaves * a.lds_priv_bytes;
  hipLaunchKernelGGL(reset_count_kernel, dim3(1), dim3(1), 0, stream, exc.d_count);
  // compile-time selections for DC + k AC, k in {1, 2, 5, 9}; any other mask at run time
  switch (g.mask) {
    case (1ull << 2) - 1: return launch_frag_mp<MaskPrefix<2>>(ds, a, lds, stream);
    case (1ull << 3) - 1: return launch_frag_mp<MaskPrefix<3>>(ds, a, lds, stream);
    case (1ull << 6) - 1: return launch_frag_mp<MaskPrefix<6>>(ds, a, lds, stream);
    case (1ull << 10) - 1: return launch_frag_mp<MaskPrefix<10>>(ds, a, lds, stream);
    default: return launch_frag_mp<MaskRuntime>(ds, a, lds, stream);
  }
}

int launch_defrag_fp32(const DeviceState &ds, const Geom &g, const float *pub, const uint8_t *priv,
                       const sf_exceptions &exc, const AesArgs &aes, uint8_t *pix, uint32_t *status,
                       hipStream_t stream) {
  DefragKernelArgs a;
  a.g = tile_geom(g, nullptr);
  a.in.pix_out = pix;
  a.in.pub = pub;
  a.in.priv = priv;
  a.aes_t0 = ds.d_aes_t0;
  a.aes = aes;
  a.K = host_tables().dct;
  a.lds_priv_bytes = lds_priv_bytes(g);
  const size_t lds = (size_t)kWaves * a.lds_priv_bytes;
  int rc;
  switch (g.mask) {
    case (1ull << 2) - 1: rc = launch_defrag_mp<MaskPrefix<2>>(ds, a, lds, stream); break;
    case (1ull << 3) - 1: rc = launch_defrag_mp<MaskPrefix<3>>(ds, a, lds, stream); break;
    case (1ull << 6) - 1: rc = launch_defrag_mp<MaskPrefix<6>>(ds, a, lds, stream); break;
    case (1ull << 10) - 1: rc = launch_defrag_mp<MaskPrefix<10>>(ds, a, lds, stream); break;
    default: rc = launch_defrag_mp<MaskRuntime>(ds, a, lds, stream); break;
  }
  if (rc) return rc;
  hipLaunchKernelGGL(apply_exceptions_kernel, dim3(64), dim3(256), 0, stream, exc.d_count, exc.d_index,
                     exc.d_value, exc.capacity, pix, (uint32_t)(g.nb * 64u), status);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SF_OK : hip_fail(e, "apply_exceptions launch");
}

}  // namespace sf
