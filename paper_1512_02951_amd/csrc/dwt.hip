// Wavelet variant of the selective encryption (report Sec. 6.8-6.9): the
// LeGall 5/3 integer lifting (Eqs. (1)-(2)) applied twice on every 8x8 block,
// rows then columns, the second level on the 4x4 low-low quarter; the 2x2
// second-level low-low corner (4 of 64 coefficients, Sec. 6.9.3) is the
// private fragment (int16, AES-128-CTR), the other 60 coefficients the public
// fragment (int16).  Integer lifting maps integers to integers and its
// inverse undoes it step by step, so defragmentation is exact by
// construction: no certificate and no residual.
//
// One wavefront per tile of 64 blocks, one block per lane (as the DCT form);
// samples enter as x - 128 (Sec. 6.9.4).  1-D lifting on n = 8 or 4 samples,
// whole-sample symmetric extension (x(-1) = x(1), x(n) = x(n - 2)):
//   d(i) = x(2i+1) - floor((x(2i) + x(2i+2)) / 2)
//   s(i) = x(2i)   + floor((d(i-1) + d(i) + 2) / 4)
// floor of a signed division by 2 or 4 is an arithmetic shift.
#include "plain_tile.h"

namespace sf {
namespace {

constexpr int kWaves = 2;
constexpr int kThreads = 64 * kWaves;
constexpr uint32_t kDwtPriv = 4, kDwtPub = 60;

// Forward 1-D lifting of v[0..N-1] at stride S inside a (8x8) array: writes
// the N/2 low outputs then the N/2 high outputs back in place.
template <int N, int S>
__device__ __forceinline__ void lift_fwd(int32_t *v) {
  constexpr int Hn = N / 2;
  int32_t x[N], d[Hn], s[Hn];
#pragma unroll
  for (int i = 0; i < N; ++i) x[i] = v[i * S];
#pragma unroll
  for (int i = 0; i < Hn; ++i) {
    const int32_t right = 2 * i + 2 < N ? x[2 * i + 2] : x[N - 2];
    d[i] = x[2 * i + 1] - ((x[2 * i] + right) >> 1);
  }
#pragma unroll
  for (int i = 0; i < Hn; ++i) s[i] = x[2 * i] + (((i > 0 ? d[i - 1] : d[0]) + d[i] + 2) >> 2);
#pragma unroll
  for (int i = 0; i < Hn; ++i) {
    v[i * S] = s[i];
    v[(Hn + i) * S] = d[i];
  }
}

template <int N, int S>
__device__ __forceinline__ void lift_inv(int32_t *v) {
  constexpr int Hn = N / 2;
  int32_t s[Hn], d[Hn], e[Hn];
#pragma unroll
  for (int i = 0; i < Hn; ++i) {
    s[i] = v[i * S];
    d[i] = v[(Hn + i) * S];
  }
#pragma unroll
  for (int i = 0; i < Hn; ++i) e[i] = s[i] - (((i > 0 ? d[i - 1] : d[0]) + d[i] + 2) >> 2);
#pragma unroll
  for (int i = 0; i < Hn; ++i) {
    const int32_t right = i + 1 < Hn ? e[i + 1] : e[Hn - 1];
    v[(2 * i) * S] = e[i];
    v[(2 * i + 1) * S] = d[i] + ((e[i] + right) >> 1);
  }
}

// One 2-D level on the n x n top-left corner of the 8x8 array a (row-major).
template <int N>
__device__ __forceinline__ void level_fwd(int32_t (&a)[64]) {
  static_for<0, N>([&](auto rc) { lift_fwd<N, 1>(&a[8 * decltype(rc)::value]); });
  static_for<0, N>([&](auto cc) { lift_fwd<N, 8>(&a[decltype(cc)::value]); });
}

template <int N>
__device__ __forceinline__ void level_inv(int32_t (&a)[64]) {
  static_for<0, N>([&](auto cc) { lift_inv<N, 8>(&a[decltype(cc)::value]); });
  static_for<0, N>([&](auto rc) { lift_inv<N, 1>(&a[8 * decltype(rc)::value]); });
}

// Fragment positions: private (0,0), (0,1), (1,0), (1,1); public the other
// 60 in row-major order.
__device__ __forceinline__ constexpr bool dwt_private(int p) { return p == 0 || p == 1 || p == 8 || p == 9; }
__device__ __forceinline__ constexpr int dwt_rank(int p) {
  if (dwt_private(p)) return p == 0 ? 0 : p == 1 ? 1 : p == 8 ? 2 : 3;
  int r = 0;
  for (int q = 0; q < p; ++q) r += dwt_private(q) ? 0 : 1;
  return r;
}

struct DwtArgs {
  TileGeom g;
  int16_t *pub;        // frag output / defrag input
  uint8_t *priv;       // frag output / defrag input (ciphertext when enc)
  uint8_t *pix_out;    // defrag output
  const uint32_t *aes_t0;
  AesArgs aes;
};

__global__ __launch_bounds__(kThreads) void dwt_frag_kernel(DwtArgs a) {
  __shared__ AesLds s_aes;
  __shared__ __attribute__((aligned(16))) uint8_t s_priv[kWaves][2 * kDwtPriv * 64];
  const int lane = threadIdx.x & 63;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (a.aes.enabled) aes_load_tables(s_aes, a.aes_t0, a.aes.key, threadIdx.x, kThreads);
  __syncthreads();
  uint8_t *lp = s_priv[wave];
  const TileGeom &g = a.g;
  for (uint32_t t = blockIdx.x * kWaves + wave; t < g.ntiles; t += gridDim.x * kWaves) {
    const TileLane L = tile_lane(g, t, lane);
    const bool valid = L.valid != 0u;
    uint32_t xs[16];
    load_block(g, L, xs);
    int32_t c[64];
    static_for<0, 64>([&](auto pc) {
      constexpr int p = decltype(pc)::value;
      c[p] = (int32_t)byte_of(xs, p) - 128;
    });
    level_fwd<8>(c);
    level_fwd<4>(c);
    const uint32_t nt = L.nt;
    const __amdgpu_buffer_rsrc_t pub_rs = buffer_rsrc(a.pub + L.b0 * kDwtPub, kDwtPub * nt * 2u);
    static_for<0, 64>([&](auto pc) {
      constexpr int p = decltype(pc)::value;
      constexpr int j = dwt_rank(p);
      if constexpr (dwt_private(p)) {
        if (valid) *reinterpret_cast<int16_t *>(lp + 2u * (j * nt + lane)) = (int16_t)c[p];
      } else {
        if (valid)
          __builtin_amdgcn_raw_buffer_store_b16((uint16_t)c[p], pub_rs, lane * 2, (int)(j * nt * 2u), kNonTemporal);
      }
    });
    wave_lds_sync();
    tile_ctr_store(lp, a.priv + L.b0 * kDwtPriv * 2u, 2u * kDwtPriv * nt, lane, s_aes, a.aes.enabled, a.aes.ctr_hi,
                   a.aes.ctr_lo, L.b0 * kDwtPriv / 8u);
    wave_lds_sync();
  }
}

__global__ __launch_bounds__(kThreads) void dwt_defrag_kernel(DwtArgs a) {
  __shared__ AesLds s_aes;
  __shared__ __attribute__((aligned(16))) uint8_t s_priv[kWaves][2 * kDwtPriv * 64];
  const int lane = threadIdx.x & 63;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (a.aes.enabled) aes_load_tables(s_aes, a.aes_t0, a.aes.key, threadIdx.x, kThreads);
  __syncthreads();
  uint8_t *lp = s_priv[wave];
  const TileGeom &g = a.g;
  for (uint32_t t = blockIdx.x * kWaves + wave; t < g.ntiles; t += gridDim.x * kWaves) {
    const TileLane L = tile_lane(g, t, lane);
    const bool valid = L.valid != 0u;
    const uint32_t nt = L.nt;
    int32_t c[64];
    const __amdgpu_buffer_rsrc_t pub_rs = buffer_rsrc(a.pub + L.b0 * kDwtPub, kDwtPub * nt * 2u);
    const int voff = valid ? lane * 2 : 0;  // lanes past the tile's end read lane 0's values, never stored
    static_for<0, 64>([&](auto pc) {
      constexpr int p = decltype(pc)::value;
      constexpr int j = dwt_rank(p);
      if constexpr (!dwt_private(p))
        c[p] = (int32_t)(int16_t)__builtin_amdgcn_raw_buffer_load_b16(pub_rs, voff, (int)(j * nt * 2u), kNonTemporal);
    });
    tile_ctr_load(lp, a.priv + L.b0 * kDwtPriv * 2u, 2u * kDwtPriv * nt, lane, s_aes, a.aes.enabled, a.aes.ctr_hi,
                  a.aes.ctr_lo, L.b0 * kDwtPriv / 8u);
    wave_lds_sync();
    static_for<0, 64>([&](auto pc) {
      constexpr int p = decltype(pc)::value;
      constexpr int j = dwt_rank(p);
      if constexpr (dwt_private(p))
        c[p] = valid ? (int32_t) * reinterpret_cast<const int16_t *>(lp + 2u * (j * nt + lane)) : 0;
    });
    wave_lds_sync();
    level_inv<4>(c);
    level_inv<8>(c);
    if (valid) {
      uint8_t *px = a.pix_out + L.org;
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        uint32_t w[2] = {0u, 0u};
#pragma unroll
        for (int i = 0; i < 8; ++i) w[i >> 2] |= (uint32_t)((c[8 * r + i] + 128) & 0xff) << (8 * (i & 3));
        __builtin_nontemporal_store(((uint64_t)w[1] << 32) | w[0], reinterpret_cast<uint64_t *>(px + (size_t)r * g.W));
      }
    }
  }
}

int dwt_grid(uint32_t ntiles) {
  const uint64_t need = ((uint64_t)ntiles + kWaves - 1) / kWaves;
  return (int)(need < 0x7fffffffu ? need : 0x7fffffffu);
}

}  // namespace

int launch_dwt_frag(const DeviceState &ds, const Geom &g, const uint8_t *pix, int16_t *pub, uint8_t *priv,
                    const AesArgs &aes, hipStream_t stream) {
  DwtArgs a{};
  a.g = tile_geom(g, pix);
  a.pub = pub;
  a.priv = priv;
  a.aes_t0 = ds.d_aes_t0;
  a.aes = aes;
  hipLaunchKernelGGL(dwt_frag_kernel, dim3(dwt_grid(g.ntiles)), dim3(kThreads), 0, stream, a);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SF_OK : hip_fail(e, "wavelet frag launch");
}

int launch_dwt_defrag(const DeviceState &ds, const Geom &g, const int16_t *pub, const uint8_t *priv,
                      const AesArgs &aes, uint8_t *pix, hipStream_t stream) {
  DwtArgs a{};
  a.g = tile_geom(g, nullptr);
  a.pub = const_cast<int16_t *>(pub);
  a.priv = const_cast<uint8_t *>(priv);
  a.pix_out = pix;
  a.aes_t0 = ds.d_aes_t0;
  a.aes = aes;
  hipLaunchKernelGGL(dwt_defrag_kernel, dim3(dwt_grid(g.ntiles)), dim3(kThreads), 0, stream, a);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SF_OK : hip_fail(e, "wavelet defrag launch");
}

}  // namespace sf
