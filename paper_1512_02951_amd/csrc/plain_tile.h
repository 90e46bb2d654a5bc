// Per-tile bodies of the plain (FP32) form, shared by the single-image
// kernels (plain.hip) and the batched persistent kernel (batch.hip).
//
// A tile is 64 consecutive 8x8 blocks of one image, processed by one
// wavefront with one block per lane.
//
// frag: coalesced 8-byte row loads (one row load of a wave covers 512
// contiguous bytes when the tile lies in one block row), FP32 DCT butterflies
// in registers, integer private quantiser on the packed pixel words (int8 dot
// products), zigzag split (compile-time for "DC + k AC" selections,
// wave-uniform branches for any other mask), public coefficients stored
// straight into the tile-interleaved layout (each store instruction writes
// 256 contiguous bytes), exactness certificate per block and, for the rare
// waves whose certificate does not rule out a miss, the reconstruction check
// (the stored values go through the very routine defrag uses; samples that
// would not round back go to the tile's exception slots, positions found with
// a wave prefix sum), private integers staged in LDS and AES-128-CTR encrypted
// 16 bytes per lane with coalesced 16-byte stores.
//
// defrag: decrypt the tile's private bytes into LDS, gather private and
// public values in zigzag order, inverse DCT, round half to even, clamp,
// coalesced 8-byte row stores, then the tile's exceptions (if any) are
// written by the lanes owning their blocks.
#pragma once

#include "sf_internal.h"

namespace sf {

// Unsigned division by an invariant divisor d >= 1 as a multiply-high and
// shifts (Granlund and Montgomery, "Division by invariant integers using
// multiplication", PLDI 1994, Sec. 4): with l = ceil(log2 d) and
// m = floor(2^32 (2^l - d) / d) + 1 (which fits 32 bits), every 32-bit n has
// n / d = (t + ((n - t) >> s1)) >> s2, t = mulhi(m, n), s1 = min(l, 1),
// s2 = max(l - 1, 0).  The three words are wave-uniform kernel arguments, so
// no vector register holds a reciprocal.
struct UDiv {
  uint32_t m, s1, s2;
};

inline UDiv udiv_magic(uint32_t d) {
  uint32_t l = 0;
  while (l < 32u && (1ull << l) < (uint64_t)d) ++l;
  UDiv u;
  u.m = (uint32_t)(((1ull << 32) * ((1ull << l) - d)) / d + 1u);
  u.s1 = l ? 1u : 0u;
  u.s2 = l ? l - 1u : 0u;
  return u;
}

__device__ __forceinline__ uint32_t udiv(uint32_t n, const UDiv &u) {
  const uint32_t t = __umulhi(u.m, n);
  return (t + ((n - t) >> u.s1)) >> u.s2;
}

struct TileGeom {
  const uint8_t *pix;
  uint32_t H, W, Bx, By;
  uint64_t nb;
  uint32_t ntiles, npriv, npub;
  UDiv div_plane, div_bx;  // division by Bx * By and by Bx
  uint64_t mask;
};

inline TileGeom tile_geom(const Geom &g, const uint8_t *pix) {
  TileGeom t;
  t.pix = pix;
  t.H = g.H;
  t.W = g.W;
  t.Bx = g.Bx;
  t.By = g.By;
  t.nb = g.nb;
  t.ntiles = g.ntiles;
  t.npriv = g.npriv;
  t.npub = g.npub;
  t.mask = g.mask;
  t.div_plane = udiv_magic(g.Bx * g.By);
  t.div_bx = udiv_magic(g.Bx);
  return t;
}

// Exception slots of one image (see sf_exception_bytes): per tile a uint16
// count, then per_tile uint16 positions (block-in-tile * 64 + sample-in-block)
// and per_tile uint8 values.
struct ExcSlots {
  uint16_t *count;
  uint16_t *pos;
  uint8_t *val;
  uint32_t per_tile;
  uint32_t check;  // 0: this selection never needs exceptions (nothing read or written)
};

// Slots of an image's exception buffer (plain.hip); check = 0 when the
// selection can never need exceptions.
ExcSlots exc_slots(const Geom &g, const sf_exceptions *exc);

struct FragOut {
  float *pub;
  uint8_t *priv;
  ExcSlots exc;
  uint32_t *status;
  const uint32_t *q2;
  float cert_thr;  // a block whose certificate reaches this is checked sample by sample
};

struct DefragIn {
  uint8_t *pix_out;
  const float *pub;
  const uint8_t *priv;
  ExcSlots exc;
};

// Selection policies.  MaskPrefix<NP>: zigzag positions 0..NP-1 are private
// (DC + (NP-1) AC), resolved at compile time.  MaskRuntime: any mask, one
// wave-uniform branch per zigzag position.
template <int NP>
struct MaskPrefix {
  static constexpr bool kStatic = true;
  static constexpr int kNPriv = NP;
};
struct MaskRuntime {
  static constexpr bool kStatic = false;
  static constexpr int kNPriv = -1;
};

// Cache policy of the public-fragment buffer accesses: streaming
// (non-temporal).  Every byte is touched once per call, and measured on the
// 4096^2 RGB round trip this beats the default policy (frag 57 -> 50 us).
constexpr int kNonTemporal = 2;

// Raw buffer resource over [base, base + bytes): per-tile fragment regions
// are addressed as base (SGPRs) + lane offset (one VGPR) + coefficient offset
// (an SGPR), so no 64-bit per-lane address arithmetic is spent per access.
// Word 3 selects 32-bit untyped data.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(const void *base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, 0x00020000);
}

__device__ __forceinline__ uint64_t opaque_u64(uint64_t v) {
  uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
  asm volatile("" : "+s"(lo), "+s"(hi));
  return (uint64_t)lo | ((uint64_t)hi << 32);
}

// Calls fpriv(integral_constant<n>, rank) or fpub(integral_constant<n>, rank)
// for every zigzag position, n = natural index of the position.
template <class MP, class FP, class FQ>
__device__ __forceinline__ void for_each_coef(uint64_t mask, FP &&fpriv, FQ &&fpub) {
  static_for<0, 64>([&](auto zc) {
    constexpr int z = decltype(zc)::value;
    constexpr int n = kZigZag.nat[z];
    if constexpr (MP::kStatic) {
      if constexpr (z < MP::kNPriv) fpriv(std::integral_constant<int, n>{}, (uint32_t)z);
      else fpub(std::integral_constant<int, n>{}, (uint32_t)(z - MP::kNPriv));
    } else {
      const uint32_t pr = (uint32_t)__builtin_popcountll(mask & ((1ull << z) - 1ull));
      if ((mask >> z) & 1u) fpriv(std::integral_constant<int, n>{}, pr);
      else fpub(std::integral_constant<int, n>{}, (uint32_t)z - pr);
    }
  });
}

// Sample offset of row 0 of block b within the image.
__device__ __forceinline__ uint32_t block_origin(const TileGeom &g, uint32_t b) {
  const uint32_t c = udiv(b, g.div_plane), rem = b - c * (g.Bx * g.By);
  const uint32_t by = udiv(rem, g.div_bx), bx = rem - by * g.Bx;
  return c * g.H * g.W + by * 8u * g.W + bx * 8u;
}

// Exclusive prefix sum over the 64 lanes of a wave (and the total).  Called
// by the whole wave.
__device__ __forceinline__ uint32_t wave_exclusive_scan(uint32_t v, int, uint32_t &total) {
  const uint32_t lane = fresh_lane();
  uint32_t incl = v;
#pragma unroll
  for (uint32_t d = 1; d < 64; d <<= 1) {
    const uint32_t o = (uint32_t)__builtin_amdgcn_ds_bpermute((int)((lane - d) << 2), (int)incl);
    if (lane >= d) incl += o;
  }
  total = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
  return incl - v;
}

// Orders a wave's LDS writes before its later LDS reads by other lanes (LDS
// requests of one wave are served in order; this only stops the compiler
// from moving them).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint32_t byte_of(const uint32_t (&w)[16], int p) { return (w[p / 4] >> (8 * (p % 4))) & 0xffu; }

// ---------------------------------------------------------------------------
// Private integers of up to 16 AC coefficients of a tile as int8 matrix
// products on the matrix cores (v_mfma_i32_16x16x64_i8): M = 16 blocks,
// K = the block's 64 samples minus 128 (signed bytes), N = the private AC
// coefficients.  One product per signed-byte limb of Bq, combined in the
// accumulator as ((D_h 2^8) + D_m) 2^8 + D_l, then + 128 sum_p Bq: the same
// integer acc as q2_acc (all arithmetic modulo 2^32, exact result in range).
// Lane l holds A row l % 16 and B column l % 16 over samples 16 (l / 16) ..
// 16 (l / 16) + 15; D row 4 (l / 16) + r (r = 0..3), column l % 16.  Pixels
// reach the A layout through LDS (80-byte rows: conflict-free 16-byte reads);
// accumulators return to the lane owning the block through LDS rows of 272
// bytes per coefficient.
typedef int q2v4 __attribute__((ext_vector_type(4)));
typedef unsigned int q2u4 __attribute__((ext_vector_type(4)));
constexpr uint32_t kQ2PixStride = 80;
constexpr uint32_t kQ2AccStride = 272;
constexpr uint32_t kQ2StageBytes = 64 * kQ2PixStride;  // also holds 16 rows of 272
constexpr int kQ2MfmaMaxAc = 16;
static_assert(kQ2StageBytes >= kQ2MfmaMaxAc * kQ2AccStride, "stage too small");

struct Q2Operands {
  q2v4 b[3];     // limbs l, m, h of column lane % 16, samples 16 (lane / 16) + 0..15
  uint32_t bias;  // 128 sum_p Bq of that column
};

// Natural index of the a-th private AC coefficient (zigzag order), -1 if none.
template <class MP>
__device__ __forceinline__ int private_ac(uint64_t mask, int a) {
  int n = -1, seen = 0;
  static_for<1, 64>([&](auto zc) {
    constexpr int z = decltype(zc)::value;
    bool priv;
    if constexpr (MP::kStatic) priv = z < MP::kNPriv;
    else priv = (mask >> z) & 1u;
    if (priv) {
      if (seen == a) n = kZigZag.nat[z];
      ++seen;
    }
  });
  return n;
}

__device__ __forceinline__ Q2Operands q2_operands(const uint32_t *q2, int n, int lane) {
  Q2Operands o;
  const int g = lane >> 4;
#pragma unroll
  for (int L = 0; L < 3; ++L)
#pragma unroll
    for (int j = 0; j < 4; ++j) o.b[L][j] = n >= 0 ? (int)q2[n * kQ2RowWords + 16 * L + 4 * g + j] : 0;
  o.bias = n >= 0 ? q2[n * kQ2RowWords + 48] : 0u;
  return o;
}

// The three steps of q2_mfma, for callers that read more of the staged
// pixels between them: (1) the lane's block (signed bytes) into its 80-byte
// LDS row; (2) after wave_lds_sync(), the lane's A operands; (3) after a
// second wave_lds_sync(), the products, written over the staged pixels.
__device__ __forceinline__ void q2_stage_pixels(const uint32_t (&xs)[16], int lane, uint8_t *stage) {
  uint4 *own = reinterpret_cast<uint4 *>(stage + lane * kQ2PixStride);
#pragma unroll
  for (int j = 0; j < 4; ++j) own[j] = make_uint4(xs[4 * j], xs[4 * j + 1], xs[4 * j + 2], xs[4 * j + 3]);
}

__device__ __forceinline__ void q2_read_a(int lane, const uint8_t *stage, q2v4 (&A)[4]) {
  const uint8_t *src = stage + (lane & 15) * kQ2PixStride + 16 * (lane >> 4);
#pragma unroll
  for (int bg = 0; bg < 4; ++bg) A[bg] = *reinterpret_cast<const q2v4 *>(src + 16 * bg * kQ2PixStride);
}

__device__ __forceinline__ void q2_products(const q2v4 (&A)[4], int lane, uint8_t *stage, const Q2Operands &Qs) {
  uint8_t *dst = stage + (lane & 15) * kQ2AccStride + 16 * (lane >> 4);
  const Q2Operands Q = Qs;  // from LDS: not held in registers between tiles
#pragma unroll
  for (int bg = 0; bg < 4; ++bg) {
    q2v4 c = {0, 0, 0, 0};
    c = __builtin_amdgcn_mfma_i32_16x16x64_i8(A[bg], Q.b[2], c, 0, 0, 0);
    c = (q2v4)((q2u4)c << 8u);
    c = __builtin_amdgcn_mfma_i32_16x16x64_i8(A[bg], Q.b[1], c, 0, 0, 0);
    c = (q2v4)((q2u4)c << 8u);
    c = __builtin_amdgcn_mfma_i32_16x16x64_i8(A[bg], Q.b[0], c, 0, 0, 0);
    c = (q2v4)((q2u4)c + Q.bias);
    *reinterpret_cast<q2v4 *>(dst + 64 * bg) = c;
  }
}

// xs: the lane's block as signed bytes (samples - 128); Qs: the lane's B
// operand (kept in LDS by the kernel).  Leaves acc of AC index a for block
// `lane` at stage + a * kQ2AccStride + 4 lane; the caller issues
// wave_lds_sync() before reading it.
__device__ __forceinline__ void q2_mfma(const uint32_t (&xs)[16], int lane, uint8_t *stage, const Q2Operands &Qs) {
  q2_stage_pixels(xs, lane, stage);
  wave_lds_sync();
  q2v4 A[4];
  q2_read_a(lane, stage, A);
  wave_lds_sync();
  q2_products(A, lane, stage, Qs);
}

__device__ __forceinline__ int32_t q2_mfma_acc(const uint8_t *stage, uint32_t a, int lane) {
  return reinterpret_cast<const int32_t *>(stage + a * kQ2AccStride)[lane];
}

// Keystream word c (state column c) of counter block ctr_first + i.
__device__ __forceinline__ uint32_t ctr_word_quad(const AesLds &s_aes, uint64_t ctr_hi, uint64_t ctr_lo,
                                                  uint64_t i, uint32_t c) {
  uint32_t w0, w1, w2, w3;
  aes_counter(ctr_hi, ctr_lo, i, w0, w1, w2, w3);
  const uint32_t w = c == 0 ? w0 : c == 1 ? w1 : c == 2 ? w2 : w3;
  return aes_encrypt_quad(w, c, s_aes);
}

// AES-CTR over the tile's private byte range [0, tbytes) held in LDS at lp;
// writes the result to gp.  ctr_first = index of the tile's first AES block
// in the fragment's counter sequence.  Whole passes of 64 blocks take one
// block per lane; a last pass of at most 16 blocks takes one block per quad
// of lanes (aes_encrypt_quad), one 4-byte word per lane.
__device__ __forceinline__ void tile_ctr_store(uint8_t *lp, uint8_t *gp, uint32_t tbytes, int lane, const AesLds &s_aes,
                                               uint32_t enc, uint64_t ctr_hi, uint64_t ctr_lo, uint64_t ctr_first) {
  const uint32_t nblk = (tbytes + 15u) / 16u;
  const uint32_t rem = nblk & 63u;
  const uint32_t nrow = enc && rem != 0u && rem <= 16u ? nblk - rem : nblk;  // wave-uniform
  for (uint32_t i = lane; i < nrow; i += 64) {
    uint4 v = *reinterpret_cast<const uint4 *>(lp + 16u * i);
    if (enc) {
      uint32_t w0, w1, w2, w3;
      aes_counter(ctr_hi, ctr_lo, ctr_first + i, w0, w1, w2, w3);
      aes_encrypt(w0, w1, w2, w3, s_aes);
      v.x ^= w0;
      v.y ^= w1;
      v.z ^= w2;
      v.w ^= w3;
    }
    if (16u * i + 16u <= tbytes) {
      *reinterpret_cast<uint4 *>(gp + 16u * i) = v;
    } else {  // final, partial AES block of the fragment: bytes via LDS
      *reinterpret_cast<uint4 *>(lp + 16u * i) = v;
      for (uint32_t j = 16u * i; j < tbytes; ++j) gp[j] = lp[j];
    }
  }
  if (nrow != nblk) {
    const uint32_t ln = fresh_lane();
    const uint32_t i = nrow + (ln >> 2), c = ln & 3u, o = 16u * i + 4u * c;
    uint32_t v = 0u;
    if (i < nblk) v = *reinterpret_cast<const uint32_t *>(lp + o);
    v ^= ctr_word_quad(s_aes, ctr_hi, ctr_lo, ctr_first + i, c);  // every lane: quad permutes
    if (o + 4u <= tbytes) {
      *reinterpret_cast<uint32_t *>(gp + o) = v;
    } else if (o < tbytes) {  // final, partial word of the fragment: bytes via LDS
      *reinterpret_cast<uint32_t *>(lp + o) = v;
      for (uint32_t j = o; j < tbytes; ++j) gp[j] = lp[j];
    }
  }
}

// Inverse of tile_ctr_store: global [0, tbytes) -> decrypted bytes in LDS.
__device__ __forceinline__ void tile_ctr_load(uint8_t *lp, const uint8_t *gp, uint32_t tbytes, int lane,
                                              const AesLds &s_aes, uint32_t enc, uint64_t ctr_hi, uint64_t ctr_lo,
                                              uint64_t ctr_first) {
  const uint32_t nblk = (tbytes + 15u) / 16u;
  const uint32_t rem = nblk & 63u;
  const uint32_t nrow = enc && rem != 0u && rem <= 16u ? nblk - rem : nblk;  // wave-uniform
  for (uint32_t i = lane; i < nrow; i += 64) {
    uint4 v;
    if (16u * i + 16u <= tbytes) {
      v = *reinterpret_cast<const uint4 *>(gp + 16u * i);
    } else {  // never read past the end of the fragment
      for (uint32_t j = 16u * i; j < 16u * i + 16u; ++j) lp[j] = j < tbytes ? gp[j] : (uint8_t)0;
      v = *reinterpret_cast<const uint4 *>(lp + 16u * i);
    }
    if (enc) {
      uint32_t w0, w1, w2, w3;
      aes_counter(ctr_hi, ctr_lo, ctr_first + i, w0, w1, w2, w3);
      aes_encrypt(w0, w1, w2, w3, s_aes);
      v.x ^= w0;
      v.y ^= w1;
      v.z ^= w2;
      v.w ^= w3;
    }
    *reinterpret_cast<uint4 *>(lp + 16u * i) = v;
  }
  if (nrow != nblk) {
    const uint32_t ln = fresh_lane();
    const uint32_t i = nrow + (ln >> 2), c = ln & 3u, o = 16u * i + 4u * c;
    uint32_t v = 0u;
    if (o + 4u <= tbytes) {
      v = *reinterpret_cast<const uint32_t *>(gp + o);
    } else if (o < tbytes) {  // never read past the end of the fragment
      for (uint32_t j = 0; j < 4u; ++j) v |= (o + j < tbytes ? (uint32_t)gp[o + j] : 0u) << (8u * j);
    }
    v ^= ctr_word_quad(s_aes, ctr_hi, ctr_lo, ctr_first + i, c);  // every lane: quad permutes
    if (i < nblk) *reinterpret_cast<uint32_t *>(lp + o) = v;
  }
}

// Blocks of tile t: number of blocks and this lane's block origin.
struct TileLane {
  uint64_t b0;   // first block of the tile
  uint32_t nt;   // blocks in the tile (64 except for the last tile)
  uint32_t valid;  // this lane holds a block (0 or 1)
  uint32_t org;  // sample offset of the lane's block
};

__device__ __forceinline__ TileLane tile_lane(const TileGeom &g, uint32_t t, int lane) {
  TileLane L;
  L.b0 = (uint64_t)t * 64u;
  L.nt = (uint32_t)min<uint64_t>(64u, g.nb - L.b0);
  L.valid = (uint32_t)lane < L.nt ? 1u : 0u;
  L.org = L.valid ? block_origin(g, (uint32_t)L.b0 + lane) : 0u;
  return L;
}

// The lane's 8x8 block as 16 words (row r = words 2r, 2r+1), zero if no block.
__device__ __forceinline__ void load_block(const TileGeom &g, const TileLane &L, uint32_t (&xs)[16]) {
  if (L.valid) {
    const uint8_t *p = g.pix + L.org;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const uint2 v = *reinterpret_cast<const uint2 *>(p + (size_t)r * g.W);
      xs[2 * r] = v.x;
      xs[2 * r + 1] = v.y;
    }
  } else {
#pragma unroll
    for (int w = 0; w < 16; ++w) xs[w] = 0u;
  }
}

struct NoPrefetch {
  __device__ void operator()() const {}
};

// True for compile-time selections whose private positions all lie in the
// 4 x 4 low-frequency corner (u, v < 4; "DC + k AC" up to k = 9).
template <class MP>
constexpr bool corner_selection() {
  if constexpr (!MP::kStatic) {
    return false;
  } else {
    for (int z = 0; z < MP::kNPriv; ++z)
      if (kZigZag.nat[z] / 8 > 3 || kZigZag.nat[z] % 8 > 3) return false;
    return true;
  }
}

template <class MP>
constexpr bool private_nat(int n) {
  for (int z = 0; z < MP::kNPriv; ++z)
    if (kZigZag.nat[z] == n) return true;
  return false;
}

// 1-D basis value c(u) cos((2x + 1) u pi / 16) for u, x < 4 from the
// butterfly constants; b_u(7 - x) = (-1)^u b_u(x).
template <int U, int X>
__device__ __forceinline__ float basis1(const DctK &K) {
  if constexpr (U == 0) return K.s0;
  else if constexpr (U == 1) return X == 0 ? K.c1 : X == 1 ? K.c3 : X == 2 ? K.c5 : K.c7;
  else if constexpr (U == 2) return X == 0 ? K.a : X == 1 ? K.b : X == 2 ? -K.b : -K.a;
  else return X == 0 ? K.c3 : X == 1 ? -K.c7 : X == 2 ? -K.c1 : -K.c5;
}

// The inverse transform of the private rounding d (natural index n = 8u + v,
// only positions of a corner selection), sample by sample: f(p, value) for
// p = 8y + x.  Separable, with the even/odd symmetry of the 1-D basis in
// both directions; terms of public positions are left out at compile time.
template <class MP, class F>
__device__ __forceinline__ void corner_estimate(const float (&d)[64], const DctK &K, F &&f) {
  float T[4][8];  // T[u][x] = sum_v d[8u + v] b_v(x)
  static_for<0, 4>([&](auto uc) {
    constexpr int u = decltype(uc)::value;
    static_for<0, 4>([&](auto xc) {
      constexpr int x = decltype(xc)::value;
      float ev = 0.0f, od = 0.0f;
      bool he = false, ho = false;
      static_for<0, 4>([&](auto vc) {
        constexpr int v = decltype(vc)::value;
        if constexpr (private_nat<MP>(8 * u + v)) {
          float &acc = (v & 1) ? od : ev;
          bool &has = (v & 1) ? ho : he;
          acc = has ? __builtin_fmaf(d[8 * u + v], basis1<v, x>(K), acc) : d[8 * u + v] * basis1<v, x>(K);
          has = true;
        }
      });
      T[u][x] = ev + od;
      T[u][7 - x] = ev - od;
    });
  });
  static_for<0, 4>([&](auto yc) {
    constexpr int y = decltype(yc)::value;
    static_for<0, 8>([&](auto xc) {
      constexpr int x = decltype(xc)::value;
      const float ev = __builtin_fmaf(T[2][x], basis1<2, y>(K), T[0][x] * basis1<0, y>(K));
      const float od = __builtin_fmaf(T[3][x], basis1<3, y>(K), T[1][x] * basis1<1, y>(K));
      f(std::integral_constant<int, 8 * y + x>{}, ev + od);
      f(std::integral_constant<int, 8 * (7 - y) + x>{}, ev - od);
    });
  });
}

// kQ2Mfma: private AC integers from q2_mfma (at most 16 private AC
// coefficients; q2stage and Q as set up by the kernel), else from q2_acc.
// prefetch() (which may overwrite xs with the next tile's pixels) is called
// once xs is dead, before the encryption pass, so those loads are in flight
// during the rest of the tile.
template <class MP, bool kQ2Mfma = false, class PF = NoPrefetch>
__device__ __forceinline__ void frag_tile(const TileGeom &g, const FragOut &o, uint32_t t, const TileLane &L,
                                          uint32_t (&xs)[16], int lane, uint8_t *lp, const AesLds &s_aes, uint32_t enc,
                                          uint64_t ctr_hi, uint64_t ctr_lo, const DctK &K, uint8_t *q2stage = nullptr,
                                          const Q2Operands *Q = nullptr, PF &&prefetch = PF{}) {
  const uint64_t b0 = L.b0;
  const uint32_t nt = L.nt;
  const bool valid = L.valid != 0u;
  const uint64_t mask = MP::kStatic ? g.mask : opaque_u64(g.mask);

  float c[64];
  static_for<0, 64>([&](auto pc) {
    constexpr int p = decltype(pc)::value;
    c[p] = (float)byte_of(xs, p);
  });
  uint32_t S = 0;  // block sum, exact
#pragma unroll
  for (int w = 0; w < 16; ++w) S = __builtin_amdgcn_udot4(xs[w], 0x01010101u, S, false);
#pragma unroll
  for (int w = 0; w < 16; ++w) xs[w] ^= 0x80808080u;  // now pixels - 128, signed bytes

  if constexpr (kQ2Mfma) q2_mfma(xs, lane, q2stage, *Q);
  fdct8x8(c, K);
  if constexpr (kQ2Mfma) wave_lds_sync();
  const uint32_t dc_priv = MP::kStatic ? 1u : (uint32_t)(mask & 1u);

  // ---- zigzag split
  const __amdgpu_buffer_rsrc_t pub_rs = buffer_rsrc(o.pub + b0 * g.npub, g.npub * nt * 4u);
  const int pub_voff = lane * 4;
  const cu32_ptr q2 = as_const(o.q2) + opaque_zero();
  // cert = sum over private n of (|q_n - acc_n / 2^20| + E_n) * M_n bounds how far
  // the private rounding moves any reconstructed sample (table words kQ2Cert*).
  float cert = 0.0f;
  // for selections inside the 4 x 4 low-frequency corner: the signed private
  // rounding d_n = q_n - acc_n / 2^20 (exact in FP32) and sum_n E_n M_n
  float dq[64];
  float sum_em = 0.0f;
  for_each_coef<MP>(
      mask,
      [&](auto nc, uint32_t pr) {
        constexpr int n = decltype(nc)::value;
        int32_t q;
        if constexpr (n == 0) {
          q = (int32_t)((S + 3u + ((S >> 3) & 1u)) >> 3);  // round half even of S / 8
          const int32_t d = 8 * q - (int32_t)S;                // 8 (q - S/8), exact
          cert += (float)(d < 0 ? -d : d) * (0.125f * 0.125f);  // M_0 = 1/8, E_0 = 0
          dq[0] = (float)d * 0.125f;
        } else {
          const cu32_ptr row = q2 + n * kQ2RowWords;
          int32_t acc;
          if constexpr (kQ2Mfma) acc = q2_mfma_acc(q2stage, pr - dc_priv, lane);
          else acc = q2_acc(xs, row);
          q = q2_round(acc);
          const int32_t d = (int32_t)((uint32_t)q << 20) - acc;  // |d| <= 2^19
          const float e = __builtin_fmaf((float)(d < 0 ? -d : d), 0x1p-20f, __uint_as_float(row[kQ2CertE]));
          cert = __builtin_fmaf(e, __uint_as_float(row[kQ2CertM]), cert);
          if constexpr (corner_selection<MP>()) {
            dq[n] = (float)d * 0x1p-20f;
            sum_em = __builtin_fmaf(__uint_as_float(row[kQ2CertE]), __uint_as_float(row[kQ2CertM]), sum_em);
          }
        }
        if (valid) *reinterpret_cast<int16_t *>(lp + 2u * (pr * nt + lane)) = (int16_t)q;
        c[n] = (float)q;
      },
      [&](auto nc, uint32_t pu) {
        constexpr int n = decltype(nc)::value;
        if (valid)
          __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(c[n]), pub_rs, pub_voff, (int)(pu * nt * 4u), kNonTemporal);
      });

  // ---- reconstruction check on exactly the stored values, for waves holding
  // a block whose certificate does not rule out a miss
  if (o.exc.check) {
    uint32_t total = 0;
    if (__ballot(valid && cert >= o.cert_thr) != 0ull) {
      // miss bits placed with v_lshl_or_b32 (shift amount inline), which the
      // optimiser would otherwise turn into selects of 64 bit constants held
      // in registers across the whole tile loop
      uint32_t bad_lo = 0, bad_hi = 0;
      if constexpr (corner_selection<MP>()) {
        // samples whose reconstruction may miss: the signed rounding error
        // of the private part at the sample, sum_n d_n B_n(p), within
        // cert_thr - sum_n E_n M_n of 1/2 (the rest of the certificate's
        // allowance bounds everything else); these go to the exception slots
        // whether or not they would actually round wrong
        // corner_estimate gives the samples in the order g = 16 y + 2 x + s
        // (sample 8 y + x for s = 0, 8 (7 - y) + x for s = 1, y < 4); each
        // one shifts the sign of |e| - thr into a word (v_alignbit_b32), so
        // after 32 samples sample g sits at bit 31 - g % 32 of word g / 32,
        // and the bit is clear where |e| >= thr
        const float thr = o.cert_thr - sum_em;
        corner_estimate<MP>(dq, K, [&](auto pc, float e) {
          constexpr int p = decltype(pc)::value, row = p / 8, x = p % 8;
          constexpr int gg = row < 4 ? 16 * row + 2 * x : 16 * (7 - row) + 2 * x + 1;
          uint32_t &acc = gg < 32 ? bad_lo : bad_hi;
          acc = __builtin_amdgcn_alignbit(acc, __float_as_uint(__builtin_fabsf(e) - thr), 31);
        });
        bad_lo = ~bad_lo;
        bad_hi = ~bad_hi;
      } else {
        idct8x8(c, K);
#pragma unroll
        for (int w = 0; w < 16; ++w) xs[w] ^= 0x80808080u;  // back to pixel bytes
        static_for<0, 64>([&](auto pc) {
          constexpr int p = decltype(pc)::value;
          const float r = __builtin_amdgcn_fmed3f(__builtin_rintf(c[p]), 0.0f, 255.0f);
          const uint32_t miss = r != (float)byte_of(xs, p) ? 1u : 0u;
          uint32_t &acc = p < 32 ? bad_lo : bad_hi;
          asm("v_lshl_or_b32 %0, %1, %2, %0" : "+v"(acc) : "v"(miss), "i"(p & 31));
        });
      }
      uint64_t bad = (uint64_t)bad_lo | ((uint64_t)bad_hi << 32);
      if (!valid) bad = 0;
      uint32_t slot = wave_exclusive_scan((uint32_t)__builtin_popcountll(bad), lane, total);
      while (bad) {
        uint32_t p = (uint32_t)__builtin_ctzll(bad);
        bad &= bad - 1ull;
        if constexpr (corner_selection<MP>()) {  // bit of sample g (see above) -> sample
          const uint32_t gg = 32u * (p >> 5) + 31u - (p & 31u), y = gg >> 4, x = (gg >> 1) & 7u;
          p = (gg & 1u) ? 8u * (7u - y) + x : 8u * y + x;
        }
        if (slot < o.exc.per_tile) {
          const size_t e = (size_t)t * o.exc.per_tile + slot;
          o.exc.pos[e] = (uint16_t)(lane * 64 + p);
          o.exc.val[e] = g.pix[L.org + (p >> 3) * g.W + (p & 7u)];
        }
        ++slot;
      }
      if (total > o.exc.per_tile && o.status && lane == 0) atomicOr(o.status, SF_STATUS_EXC_OVERFLOW);
    }
    if (lane == 0) o.exc.count[t] = (uint16_t)(total < 65535u ? total : 65535u);
  }

  // the pixel words are dead from here on
  prefetch();

  // ---- private bytes of the tile: AES-CTR, 16 bytes per lane, coalesced
  wave_lds_sync();
  tile_ctr_store(lp, o.priv + b0 * g.npriv * 2u, 2u * g.npriv * nt, lane, s_aes, enc, ctr_hi, ctr_lo,
                 b0 * g.npriv / 8u);
  wave_lds_sync();
}

template <class MP>
__device__ __forceinline__ void defrag_tile(const TileGeom &g, const DefragIn &in, uint32_t t, const TileLane &L,
                                            int lane, uint8_t *lp, const AesLds &s_aes, uint32_t enc, uint64_t ctr_hi,
                                            uint64_t ctr_lo, const DctK &K) {
  const uint64_t b0 = L.b0;
  const uint32_t nt = L.nt;
  const bool valid = L.valid != 0u;
  const uint64_t mask = MP::kStatic ? g.mask : opaque_u64(g.mask);

  // public values first: their loads stay in flight while the private bytes
  // are decrypted
  float c[64];
  const __amdgpu_buffer_rsrc_t pub_rs = buffer_rsrc(in.pub + b0 * g.npub, g.npub * nt * 4u);
  // lanes past the tile's last block read lane 0's values (in range); their
  // results are never stored
  const int pub_voff = valid ? lane * 4 : 0;
  for_each_coef<MP>(
      mask, [&](auto, uint32_t) {},
      [&](auto nc, uint32_t pu) {
        constexpr int n = decltype(nc)::value;
        c[n] = __uint_as_float(
            __builtin_amdgcn_raw_buffer_load_b32(pub_rs, pub_voff, (int)(pu * nt * 4u), kNonTemporal));
      });
  tile_ctr_load(lp, in.priv + b0 * g.npriv * 2u, 2u * g.npriv * nt, lane, s_aes, enc, ctr_hi, ctr_lo,
                b0 * g.npriv / 8u);
  wave_lds_sync();
  for_each_coef<MP>(
      mask,
      [&](auto nc, uint32_t pr) {
        constexpr int n = decltype(nc)::value;
        c[n] = valid ? (float)*reinterpret_cast<const int16_t *>(lp + 2u * (pr * nt + lane)) : 0.0f;
      },
      [&](auto, uint32_t) {});
  wave_lds_sync();

  idct8x8(c, K);

  uint8_t *p = in.pix_out + L.org;
  if (valid) {
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      uint32_t w[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        // v_cvt_pk_u8_f32 rounds half to even and saturates to [0, 255]
        // (checked on gfx950 over the half-integers, the range edges and
        // 4096 values in [-20, 527)): one instruction per sample
        uint32_t acc = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i) acc = __builtin_amdgcn_cvt_pk_u8_f32(c[8 * r + 4 * h + i], i, acc);
        w[h] = acc;
      }
      __builtin_nontemporal_store(((uint64_t)w[1] << 32) | w[0], reinterpret_cast<uint64_t *>(p + (size_t)r * g.W));
    }
  }
  // ---- the tile's exceptions, written by the lane that stored the block
  // (same thread, later store to the same address)
  // (entries are fetched 64 at a time, one per lane, and taken in turn from
  // the lanes that hold them)
  if (in.exc.check) {
    const uint32_t n = in.exc.count[t];
    const uint32_t m = n < in.exc.per_tile ? n : in.exc.per_tile;
    for (uint32_t e0 = 0; e0 < m; e0 += 64u) {
      const uint32_t e = e0 + (uint32_t)lane;
      const size_t k = (size_t)t * in.exc.per_tile + e;
      const uint32_t pos_l = e < m ? (uint32_t)in.exc.pos[k] : 0u;
      const uint32_t val_l = e < m ? (uint32_t)in.exc.val[k] : 0u;
      const uint32_t cnt = m - e0 < 64u ? m - e0 : 64u;
      for (uint32_t i = 0; i < cnt; ++i) {
        const uint32_t pos = (uint32_t)__builtin_amdgcn_readlane((int)pos_l, (int)i);
        const uint32_t val = (uint32_t)__builtin_amdgcn_readlane((int)val_l, (int)i);
        // same cache policy as the row stores it overwrites
        if (valid && (pos >> 6) == (uint32_t)lane)
          __builtin_nontemporal_store((uint8_t)val, p + ((pos >> 3) & 7u) * g.W + (pos & 7u));
      }
    }
  }
}

}  // namespace sf
