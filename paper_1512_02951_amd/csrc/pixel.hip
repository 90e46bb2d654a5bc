// Pixel-domain fragment formats of the report: the private coefficients
// stored in 11 bits each (Sec. 6.4.3: DC unsigned, AC sign + 10-bit
// magnitude), or in the report's lossy 8-bit storage (AC sign + 7 bits,
// clamped; DC 11 bits), and the public part stored as one byte per sample in the pixel
// domain (Sec. 6.3.1, the inverse DCT of the remaining coefficients), with the
// strong level of protection (Sec. 6.3.2, Fig. 8) as an option: the 64 public
// bytes of a block XORed with the SHA-512 digest of its private integers.
//
// Everything is integer arithmetic:
//   q_j  = private integers (rule Q2, as in the DCT form);
//   R(p) = floor((sum_j q_j Bi[n_j][p] + 2^15) / 2^16), Bi = rhe(2^16 B),
//          the integer inverse of the private part (round half up: any
//          integer function of the q_j keeps the round trip exact, and this
//          one costs nothing beyond the products);
//   P(p) = (x(p) - R(p)) mod 256, which stands for the inverse DCT of the
//          remaining coefficients (x = IDCT(private) + IDCT(rest) exactly, so
//          P differs from IDCT(rest) only by how far R is from IDCT(private));
//   defrag: x(p) = (R(p) + P(p)) mod 256, exact for every selection.
//
// One wavefront per tile of 64 blocks, one block per lane.  The private AC
// integers come from the DCT form's int8 matrix-core quantiser.  R uses packed
// int16 dot products (v_dot2_i32_i16): the private integers in pairs against
// (Bi[n_2i][p], Bi[n_2i+1][p]) pairs that the host packs into the kernel
// arguments, so the table reaches the wave as scalar operands.  The 11-bit
// fields of a tile are assembled in LDS (ds_or) into one little-endian bit
// stream, then AES-128-CTR encrypted 16 bytes per lane as in the DCT form.
// SHA-512 (FIPS 180-4) runs per lane on a single message block.
#include "plain_tile.h"
#include "sha512_consts.h"

namespace sf {
namespace {

constexpr int kWaves = 2;
constexpr int kThreads = 64 * kWaves;
constexpr uint32_t kFieldBits = 11;
// LDS per wave: the largest tile stream plus one word read past the last field.
constexpr uint32_t kPixRegion = 16 * ((88 * kPixMaxPriv + 15) / 16) + 16;

struct PixArgs {
  TileGeom g;
  uint8_t *pub;       // public bytes, image layout (frag output / defrag input)
  uint8_t *priv;      // packed private bytes (ciphertext when enabled)
  uint8_t *pix_out;   // defrag output
  const uint32_t *q2;
  const uint32_t *aes_t0;
  AesArgs aes;
  uint32_t np;          // private coefficients per block
  uint32_t ac_bits;     // AC magnitude bits: 10 (11-bit fields) or 7 (8-bit fields)
  uint32_t rec_bits;    // bits per block record
  uint32_t stride;      // bytes per full tile, multiple of 16
  uint32_t last_bytes;  // bytes of the last tile
  uint8_t nat[kPixMaxPriv];  // natural index of private coefficient j (zigzag order)
  uint32_t inv[kPixMaxPriv / 2][64];  // (Bi[nat[2i]][p] & 0xffff) | Bi[nat[2i+1]][p] << 16
};

typedef short short2v __attribute__((ext_vector_type(2)));

__device__ __forceinline__ int32_t dot2(uint32_t a, uint32_t b, int32_t c) {
  return __builtin_amdgcn_sdot2(__builtin_bit_cast(short2v, a), __builtin_bit_cast(short2v, b), c, false);
}

typedef uint32_t u32x2_t __attribute__((ext_vector_type(2)));

// A 64-bit word from its halves as a register pair.  Written as
// (hi << 32) | lo, a sum of such words compiles to one add per half (the OR
// of disjoint bits becomes an add and is reassociated) plus a move.
__device__ __forceinline__ uint64_t pair64(uint32_t lo, uint32_t hi) {
  return __builtin_bit_cast(uint64_t, u32x2_t{lo, hi});
}

// 64-bit rotate right by a constant, as two v_alignbit_b32 on the halves.
template <int N>
__device__ __forceinline__ uint64_t rotr64(uint64_t x) {
  uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32);
  if constexpr (N >= 32) {
    const uint32_t t = lo;
    lo = hi;
    hi = t;
  }
  constexpr uint32_t n = N & 31;
  const uint32_t nlo = __builtin_amdgcn_alignbit(hi, lo, n), nhi = __builtin_amdgcn_alignbit(lo, hi, n);
  return pair64(nlo, nhi);
}

__device__ __forceinline__ uint64_t xor3_64(uint64_t a, uint64_t b, uint64_t c) {
  return pair64(xor3((uint32_t)a, (uint32_t)b, (uint32_t)c), xor3((uint32_t)(a >> 32), (uint32_t)(b >> 32), (uint32_t)(c >> 32)));
}

// Bitwise majority of three 64-bit words, one v_bitop3_b32 per half (truth
// table 0xE8: set where at least two inputs are set; symmetric in its inputs).
// Written as ANDs and XORs it compiles to four instructions per half.
__device__ __forceinline__ uint64_t maj3_64(uint64_t a, uint64_t b, uint64_t c) {
  const uint32_t lo = __builtin_amdgcn_bitop3_b32((uint32_t)a, (uint32_t)b, (uint32_t)c, 0xE8);
  const uint32_t hi = __builtin_amdgcn_bitop3_b32((uint32_t)(a >> 32), (uint32_t)(b >> 32), (uint32_t)(c >> 32), 0xE8);
  return pair64(lo, hi);
}

// Round constants as scalar-loadable memory for the rolled rounds 16..79.
struct Sha512Table {
  uint64_t k[80];
};
constexpr Sha512Table sha512_table() {
  Sha512Table t{};
  for (int i = 0; i < 80; ++i) t.k[i] = kSha512K[i];
  return t;
}
__constant__ Sha512Table c_sha512 = sha512_table();

// One SHA-512 round (FIPS 180-4, Sec. 6.4.2) on the working variables v[0..7]
// = a..h, addressed so that round t reads a at v[(8 - t % 8) % 8]: the
// variables rotate by renaming, never by moves.
template <int R>
__device__ __forceinline__ void sha512_round(uint64_t (&v)[8], uint64_t kw) {
  constexpr int o = (8 - (R & 7)) & 7;
  uint64_t &a = v[o], &b = v[(o + 1) & 7], &c = v[(o + 2) & 7], &d = v[(o + 3) & 7];
  uint64_t &e = v[(o + 4) & 7], &f = v[(o + 5) & 7], &g = v[(o + 6) & 7], &h = v[(o + 7) & 7];
  const uint64_t S1 = xor3_64(rotr64<14>(e), rotr64<18>(e), rotr64<41>(e));
  const uint64_t ch = (e & f) ^ (~e & g);
  const uint64_t t1 = h + S1 + ch + kw;
  const uint64_t S0 = xor3_64(rotr64<28>(a), rotr64<34>(a), rotr64<39>(a));
  const uint64_t mj = maj3_64(a, b, c);
  d += t1;
  h = t1 + S0 + mj;  // the new a
}

// SHA-512 of a message of 2 np bytes (np <= 16): the private integers as
// int16 little-endian.  One 1024-bit block: message, the 0x80 byte, zeros,
// the bit length in the last word.  Returns the digest words H[0..7].
// Rounds 0..15 are unrolled (most message words are constants there); rounds
// 16..79 run as a loop of 16 unrolled rounds that extends the schedule in
// place, which keeps the code and the live schedule words small.
template <int NP>
__device__ __forceinline__ void sha512_private(const int32_t (&q)[kPixMaxPriv], uint32_t np_rt, uint64_t (&Hout)[8]) {
  const uint32_t np = NP > 0 ? (uint32_t)NP : np_rt;
  // int16 slot s of the message; slot np holds the padding byte 0x80 (low byte)
  auto slot = [&](int s) -> uint32_t {
    if (s < kPixMaxPriv && (uint32_t)s < np) return (uint32_t)q[s] & 0xffffu;
    return (uint32_t)s == np ? 0x0080u : 0u;
  };
  auto be16 = [](uint32_t v) -> uint64_t { return (uint64_t)(((v & 0xffu) << 8) | (v >> 8)); };
  uint64_t W[16];
#pragma unroll
  for (int i = 0; i < 5; ++i)
    W[i] = (be16(slot(4 * i)) << 48) | (be16(slot(4 * i + 1)) << 32) | (be16(slot(4 * i + 2)) << 16) |
           be16(slot(4 * i + 3));
#pragma unroll
  for (int i = 5; i < 15; ++i) W[i] = 0;
  W[15] = (uint64_t)(16u * np);

  uint64_t v[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) v[i] = kSha512H0[i];
  static_for<0, 16>([&](auto tc) {
    constexpr int t = decltype(tc)::value;
    sha512_round<t>(v, kSha512K[t] + W[t]);
  });
#pragma unroll 1
  for (uint32_t base = 16; base < 80; base += 16) {
    static_for<0, 16>([&](auto rc) {
      constexpr int r = decltype(rc)::value;
      const uint64_t w15 = W[(r + 1) & 15], w2 = W[(r + 14) & 15];
      const uint64_t s0 = xor3_64(rotr64<1>(w15), rotr64<8>(w15), w15 >> 7);
      const uint64_t s1 = xor3_64(rotr64<19>(w2), rotr64<61>(w2), w2 >> 6);
      W[r] += s0 + W[(r + 9) & 15] + s1;
      sha512_round<r>(v, c_sha512.k[base + r] + W[r]);
    });
  }
#pragma unroll
  for (int i = 0; i < 8; ++i) Hout[i] = kSha512H0[i] + v[i];
}

// Digest bytes 8y .. 8y + 7 mask row y of the block: as a little-endian row
// (sample x in byte x) that is the byte-swapped digest word H[y].
__device__ __forceinline__ void row_mask(uint64_t Hy, uint32_t &lo, uint32_t &hi) {
  lo = __builtin_bswap32((uint32_t)(Hy >> 32));
  hi = __builtin_bswap32((uint32_t)Hy);
}

// R for row y of the block, packed one byte per sample (mod 256).
// inv: the pair table (PixArgs::inv) as scalar-loadable memory.  R(p) mod
// 256 is byte 2 of 2^15 + sum_j q_j Bi[n_j][p], so the rounding bias is the
// accumulators' initial value and v_perm_b32 packs the bytes.
template <int NPAIR>
__device__ __forceinline__ void recon_row(cu32_ptr inv, const uint32_t (&qp)[kPixMaxPriv / 2], uint32_t npair, int y,
                                          uint32_t &lo, uint32_t &hi) {
  int32_t acc[8];
#pragma unroll
  for (int x = 0; x < 8; ++x) acc[x] = 0x8000;
#pragma unroll
  for (int i = 0; i < kPixMaxPriv / 2; ++i) {
    if (NPAIR > 0 ? i < NPAIR : (uint32_t)i < npair) {
#pragma unroll
      for (int x = 0; x < 8; ++x) acc[x] = dot2(qp[i], inv[64 * i + 8 * y + x], acc[x]);
    }
  }
  const uint32_t *b = reinterpret_cast<const uint32_t *>(acc);
  lo = __builtin_amdgcn_perm(b[1], b[0], 0x0c0c0602u) | __builtin_amdgcn_perm(b[3], b[2], 0x06020c0cu);
  hi = __builtin_amdgcn_perm(b[5], b[4], 0x0c0c0602u) | __builtin_amdgcn_perm(b[7], b[6], 0x06020c0cu);
}

// The pair table inside this launch's kernel arguments (the kernel's only
// parameter is the PixArgs value, at offset 0 of the argument segment), plus
// an opaque zero so its loads stay inside the tile loop (hoisted out of it,
// 64 words per pair would be held, and spilled, across the loop).
__device__ __forceinline__ cu32_ptr inv_table() {
  const char __attribute__((address_space(4))) *ka =
      (const char __attribute__((address_space(4))) *)__builtin_amdgcn_kernarg_segment_ptr();
  return (cu32_ptr)(ka + offsetof(PixArgs, inv)) + opaque_zero();
}

// Field j of a record: DC (j = 0 when DC is private) takes 11 bits, every AC
// field ac_bits + 1 (sign above magnitude).
__device__ __forceinline__ uint32_t field_offset(uint32_t j, uint32_t dc, uint32_t acw) {
  return acw * j + (j > 0u ? dc * (kFieldBits - acw) : 0u);
}

__device__ __forceinline__ uint32_t tile_bytes(const PixArgs &a, uint32_t t) {
  return t + 1u == a.g.ntiles ? a.last_bytes : a.stride;
}

// NP > 0: "DC + (NP - 1) AC" selection resolved at compile time; NP = 0: any
// selection of at most kPixMaxPriv coefficients (a.nat, a.np).  The private
// AC integers come from the int8 matrix-core quantiser (at most 16 AC).
template <int NP, bool kStrong>
__global__ __launch_bounds__(kThreads) void pixel_frag_kernel(PixArgs a) {
  using MP = std::conditional_t<(NP > 0), MaskPrefix<NP>, MaskRuntime>;
  __shared__ AesLds s_aes;
  __shared__ __attribute__((aligned(16))) uint8_t s_bits[kWaves][kPixRegion];
  __shared__ __attribute__((aligned(16))) uint8_t s_stage[kWaves][kQ2StageBytes];
  __shared__ Q2Operands s_q2[64];  // B operand per lane (same for every wave)
  const int lane = threadIdx.x & 63;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (a.aes.enabled) aes_load_tables(s_aes, a.aes_t0, a.aes.key, threadIdx.x, kThreads);
  if (threadIdx.x < 64) s_q2[lane] = q2_operands(a.q2, private_ac<MP>(a.g.mask, lane & 15), lane);
  __syncthreads();
  uint8_t *lp = s_bits[wave];
  uint32_t *lw = reinterpret_cast<uint32_t *>(lp);
  uint8_t *stage = s_stage[wave];
  const TileGeom &g = a.g;
  const uint32_t np = NP > 0 ? (uint32_t)NP : a.np;
  const uint32_t npair = (np + 1u) / 2u;
  const uint32_t dc = NP > 0 ? 1u : (uint32_t)(g.mask & 1u);
  constexpr int kNPair = NP > 0 ? (NP + 1) / 2 : 0;
  for (uint32_t t = blockIdx.x * kWaves + wave; t < g.ntiles; t += gridDim.x * kWaves) {
    const TileLane L = tile_lane(g, t, lane);
    const bool valid = L.valid != 0u;
    const cu32_ptr inv = inv_table();
    for (uint32_t i = lane; i < kPixRegion / 16u; i += 64u) reinterpret_cast<uint4 *>(lp)[i] = make_uint4(0, 0, 0, 0);
    uint32_t xs[16];
    load_block(g, L, xs);
    uint32_t S = 0;
#pragma unroll
    for (int w = 0; w < 16; ++w) S = __builtin_amdgcn_udot4(xs[w], 0x01010101u, S, false);
    uint32_t xsg[16];
#pragma unroll
    for (int w = 0; w < 16; ++w) xsg[w] = xs[w] ^ 0x80808080u;  // samples - 128 as signed bytes
    q2_mfma(xsg, lane, stage, s_q2[lane]);
    wave_lds_sync();

    int32_t q[kPixMaxPriv];
#pragma unroll
    for (int j = 0; j < kPixMaxPriv; ++j) {
      q[j] = 0;
      if (NP > 0 ? j < NP : (uint32_t)j < np) {
        const int n = NP > 0 ? kZigZag.nat[j < 64 ? j : 0] : (int)a.nat[j];
        if (n == 0) q[j] = (int32_t)((S + 3u + ((S >> 3) & 1u)) >> 3);  // round half even of S / 8
        else q[j] = q2_round(q2_mfma_acc(stage, (uint32_t)j - dc, lane));
      }
    }
    // the public part uses the exact integers (packed in pairs for the
    // inverse); the fields and the strong-level hash hold the stored ones
    uint32_t qp[kPixMaxPriv / 2];
#pragma unroll
    for (int i = 0; i < kPixMaxPriv / 2; ++i) qp[i] = ((uint32_t)q[2 * i] & 0xffffu) | ((uint32_t)q[2 * i + 1] << 16);
    const int32_t lim = (1 << a.ac_bits) - 1;  // never reached at 10 bits (|AC| <= 1020)
#pragma unroll
    for (int j = 0; j < kPixMaxPriv; ++j) {
      const int n = NP > 0 ? kZigZag.nat[j < 64 ? j : 0] : (int)a.nat[j];
      if (n != 0) q[j] = max(-lim, min(lim, q[j]));
    }
    // fields into the tile's bit stream (zeroed above)
    if (valid) {
      const uint32_t base = (uint32_t)lane * a.rec_bits;
      const uint32_t acw = a.ac_bits + 1u;
#pragma unroll
      for (int j = 0; j < kPixMaxPriv; ++j) {
        if (NP > 0 ? j < NP : (uint32_t)j < np) {
          const int n = NP > 0 ? kZigZag.nat[j < 64 ? j : 0] : (int)a.nat[j];
          const uint32_t mag = (uint32_t)(q[j] < 0 ? -q[j] : q[j]);
          const uint32_t fld = n == 0 ? (uint32_t)q[j] : (mag | (q[j] < 0 ? 1u << a.ac_bits : 0u));
          const uint32_t pos = base + field_offset((uint32_t)j, dc, acw);
          const uint64_t v = (uint64_t)fld << (pos & 31u);
          atomicOr(&lw[pos >> 5], (uint32_t)v);
          if ((uint32_t)(v >> 32)) atomicOr(&lw[(pos >> 5) + 1u], (uint32_t)(v >> 32));
        }
      }
    }
    uint64_t Hm[8];
    if constexpr (kStrong) sha512_private<NP>(q, np, Hm);
    if (valid) {
      uint8_t *dst = a.pub + L.org;
#pragma unroll
      for (int y = 0; y < 8; ++y) {
        uint32_t rlo, rhi;
        recon_row<kNPair>(inv, qp, npair, y, rlo, rhi);
        uint32_t plo = bytes_sub(xs[2 * y], rlo), phi = bytes_sub(xs[2 * y + 1], rhi);
        if constexpr (kStrong) {
          uint32_t mlo, mhi;
          row_mask(Hm[y], mlo, mhi);
          plo ^= mlo;
          phi ^= mhi;
        }
        __builtin_nontemporal_store(((uint64_t)phi << 32) | plo, reinterpret_cast<uint64_t *>(dst + (size_t)y * g.W));
      }
    }
    wave_lds_sync();
    tile_ctr_store(lp, a.priv + (uint64_t)t * a.stride, tile_bytes(a, t), lane, s_aes, a.aes.enabled, a.aes.ctr_hi,
                   a.aes.ctr_lo, (uint64_t)t * (a.stride / 16u));
    wave_lds_sync();
  }
}

template <int NP, bool kStrong>
__global__ __launch_bounds__(kThreads) void pixel_defrag_kernel(PixArgs a) {
  __shared__ AesLds s_aes;
  __shared__ __attribute__((aligned(16))) uint8_t s_bits[kWaves][kPixRegion];
  const int lane = threadIdx.x & 63;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (a.aes.enabled) aes_load_tables(s_aes, a.aes_t0, a.aes.key, threadIdx.x, kThreads);
  __syncthreads();
  uint8_t *lp = s_bits[wave];
  const uint32_t *lw = reinterpret_cast<const uint32_t *>(lp);
  const TileGeom &g = a.g;
  const uint32_t np = NP > 0 ? (uint32_t)NP : a.np;
  const uint32_t npair = (np + 1u) / 2u;
  const uint32_t dc = NP > 0 ? 1u : (uint32_t)(g.mask & 1u);
  constexpr int kNPair = NP > 0 ? (NP + 1) / 2 : 0;
  for (uint32_t t = blockIdx.x * kWaves + wave; t < g.ntiles; t += gridDim.x * kWaves) {
    const TileLane L = tile_lane(g, t, lane);
    const bool valid = L.valid != 0u;
    // public rows first: their loads are in flight during the decryption
    uint32_t pw[16];
    if (valid) {
      const uint8_t *src = a.pub + L.org;
#pragma unroll
      for (int y = 0; y < 8; ++y) {
        const uint64_t v = __builtin_nontemporal_load(reinterpret_cast<const uint64_t *>(src + (size_t)y * g.W));
        pw[2 * y] = (uint32_t)v;
        pw[2 * y + 1] = (uint32_t)(v >> 32);
      }
    } else {
#pragma unroll
      for (int w = 0; w < 16; ++w) pw[w] = 0u;
    }
    tile_ctr_load(lp, a.priv + (uint64_t)t * a.stride, tile_bytes(a, t), lane, s_aes, a.aes.enabled, a.aes.ctr_hi,
                  a.aes.ctr_lo, (uint64_t)t * (a.stride / 16u));
    wave_lds_sync();
    int32_t q[kPixMaxPriv];
    const uint32_t base = (uint32_t)lane * a.rec_bits;
    const uint32_t acw = a.ac_bits + 1u;
#pragma unroll
    for (int j = 0; j < kPixMaxPriv; ++j) {
      q[j] = 0;
      if (NP > 0 ? j < NP : (uint32_t)j < np) {
        const int n = NP > 0 ? kZigZag.nat[j < 64 ? j : 0] : (int)a.nat[j];
        const uint32_t pos = base + field_offset((uint32_t)j, dc, acw);
        const uint64_t v = (uint64_t)lw[pos >> 5] | ((uint64_t)lw[(pos >> 5) + 1u] << 32);
        const uint32_t raw = (uint32_t)(v >> (pos & 31u));
        const int32_t mag = (int32_t)(raw & ((1u << a.ac_bits) - 1u));
        const int32_t val = n == 0 ? (int32_t)(raw & 0x7ffu) : (((raw >> a.ac_bits) & 1u) ? -mag : mag);
        q[j] = valid ? val : 0;
      }
    }
    wave_lds_sync();
    uint32_t qp[kPixMaxPriv / 2];
#pragma unroll
    for (int i = 0; i < kPixMaxPriv / 2; ++i) qp[i] = ((uint32_t)q[2 * i] & 0xffffu) | ((uint32_t)q[2 * i + 1] << 16);
    uint64_t Hm[8];
    if constexpr (kStrong) sha512_private<NP>(q, np, Hm);
    const cu32_ptr inv = inv_table();
    if (valid) {
      uint8_t *dst = a.pix_out + L.org;
#pragma unroll
      for (int y = 0; y < 8; ++y) {
        uint32_t plo = pw[2 * y], phi = pw[2 * y + 1];
        if constexpr (kStrong) {
          uint32_t mlo, mhi;
          row_mask(Hm[y], mlo, mhi);
          plo ^= mlo;
          phi ^= mhi;
        }
        uint32_t rlo, rhi;
        recon_row<kNPair>(inv, qp, npair, y, rlo, rhi);
        const uint32_t xlo = bytes_add(plo, rlo), xhi = bytes_add(phi, rhi);
        __builtin_nontemporal_store(((uint64_t)xhi << 32) | xlo, reinterpret_cast<uint64_t *>(dst + (size_t)y * g.W));
      }
    }
  }
}

int pix_grid(uint32_t ntiles) {
  const uint64_t need = ((uint64_t)ntiles + kWaves - 1) / kWaves;
  return (int)(need < 0x7fffffffu ? need : 0x7fffffffu);
}

// Prefix selections with a compile-time variant: DC + 2, 5 or 9 AC.
int static_np(uint64_t mask) {
  if (mask == 0x7ull) return 3;
  if (mask == 0x3full) return 6;
  if (mask == 0x3ffull) return 10;
  return 0;
}

template <int NP>
void launch_one(bool frag, bool strong, const PixArgs &a, int grid, hipStream_t stream) {
  if (frag) {
    if (strong) hipLaunchKernelGGL((pixel_frag_kernel<NP, true>), dim3(grid), dim3(kThreads), 0, stream, a);
    else hipLaunchKernelGGL((pixel_frag_kernel<NP, false>), dim3(grid), dim3(kThreads), 0, stream, a);
  } else {
    if (strong) hipLaunchKernelGGL((pixel_defrag_kernel<NP, true>), dim3(grid), dim3(kThreads), 0, stream, a);
    else hipLaunchKernelGGL((pixel_defrag_kernel<NP, false>), dim3(grid), dim3(kThreads), 0, stream, a);
  }
}

int launch_pixel(const DeviceState &ds, const Geom &g, bool frag, int flags, const uint8_t *pix, uint8_t *pub,
                 uint8_t *priv, uint8_t *pix_out, const AesArgs &aes, hipStream_t stream) {
  const bool strong = (flags & SF_LEVEL_STRONG) != 0;
  PixArgs a{};
  a.g = tile_geom(g, pix);
  a.pub = pub;
  a.priv = priv;
  a.pix_out = pix_out;
  a.q2 = ds.d_q2;
  a.aes_t0 = ds.d_aes_t0;
  a.aes = aes;
  a.np = g.npriv;
  const PixLayout lay = pixel_layout(g, flags);
  a.ac_bits = lay.ac_bits;
  a.rec_bits = lay.rec_bits;
  a.stride = lay.stride;
  a.last_bytes = lay.last_bytes;
  const HostTables &ht = host_tables();
  static constexpr ZigZag zz{};
  int j = 0;
  for (int z = 0; z < 64; ++z)
    if ((g.mask >> z) & 1u) a.nat[j++] = (uint8_t)zz.nat[z];
  for (int i = 0; i < (j + 1) / 2; ++i)
    for (int p = 0; p < 64; ++p) {
      const uint32_t lo = (uint32_t)ht.inv16[a.nat[2 * i] * 64 + p] & 0xffffu;
      const uint32_t hi = 2 * i + 1 < j ? (uint32_t)ht.inv16[a.nat[2 * i + 1] * 64 + p] : 0u;
      a.inv[i][p] = lo | (hi << 16);
    }
  const int grid = pix_grid(g.ntiles);
  switch (static_np(g.mask)) {
    case 3: launch_one<3>(frag, strong, a, grid, stream); break;
    case 6: launch_one<6>(frag, strong, a, grid, stream); break;
    case 10: launch_one<10>(frag, strong, a, grid, stream); break;
    default: launch_one<0>(frag, strong, a, grid, stream); break;
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SF_OK : hip_fail(e, frag ? "pixel frag launch" : "pixel defrag launch");
}

}  // namespace

PixLayout pixel_layout(const Geom &g, int flags) {
  PixLayout l;
  l.ac_bits = (flags & SF_STORAGE_8BIT) ? 7u : 10u;
  const uint32_t dc = (uint32_t)(g.mask & 1u);
  l.rec_bits = (l.ac_bits + 1u) * g.npriv + dc * (kFieldBits - (l.ac_bits + 1u));
  l.stride = 16u * ((8u * l.rec_bits + 15u) / 16u);
  const uint64_t nt_last = g.nb - 64ull * (g.ntiles - 1u);
  l.last_bytes = (uint32_t)((l.rec_bits * nt_last + 7u) / 8u);
  return l;
}

int launch_pixel_frag(const DeviceState &ds, const Geom &g, int flags, const uint8_t *pix, uint8_t *pub,
                      uint8_t *priv, const AesArgs &aes, hipStream_t stream) {
  return launch_pixel(ds, g, true, flags, pix, pub, priv, nullptr, aes, stream);
}

int launch_pixel_defrag(const DeviceState &ds, const Geom &g, int flags, const uint8_t *pub, const uint8_t *priv,
                        const AesArgs &aes, uint8_t *pix, hipStream_t stream) {
  return launch_pixel(ds, g, false, flags, nullptr, const_cast<uint8_t *>(pub), const_cast<uint8_t *>(priv), pix,
                      aes, stream);
}

}  // namespace sf
