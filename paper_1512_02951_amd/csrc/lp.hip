// Reduced-precision form: the 8x8 DCT and inverse DCT as 64x64 basis
// contractions on the matrix cores (v_mfma_f32_32x32x16_{f16,bf16}, FP32
// accumulation), public coefficients stored as fp16 or bf16, private
// integers exactly as in the plain form, and a residual that makes the
// round trip bit-exact: per sample r = x - clamp(round(y)), y the inverse
// transform of the stored fragments, kept as a 2-bit code (0: r = 0,
// 1: r = +1, 3: r = -1) and, for the rare samples with |r| >= 2 (code 2),
// the sample itself in the per-tile exception slots of the plain form.
// frag computes y with the same routine and operands defrag uses, so both
// see the same value bit for bit.
//
// One wavefront per tile of 64 blocks, processed as two halves of 32 blocks
// (the N dimension of the MFMA).  Lane half h (lane / 32) of the lane for
// block n of a half always holds columns 4h .. 4h + 3 of the block's eight
// rows: the pixels arrive in that layout (one 4-byte load per row), the
// forward transform takes them as its operand (K-step s: rows 2s, 2s + 1),
// the inverse transform returns the reconstruction in it (its M order is
// chosen so), and the residual compares the two word by word.  The
// forward's output (lane half h: coefficients 32 mt + 8 q + 4 h + c in
// zigzag order) is the inverse's operand as it stands: the inverse takes its
// K index in that order.  Private integers come from int8 matrix products
// (the exact rule of the plain form) on the same pixel words, rearranged
// into the int8 operand layout by two cross-lane swaps.  bf16 keeps its
// basis as a hi + lo pair (and splits the private integers, which bf16
// cannot hold exactly) so the transforms stay close to FP32 accuracy.
#include <string.h>

#include "plain_tile.h"

namespace sf {

// ---------------------------------------------------------------------------
// Host: basis operand tables in per-lane order.
namespace {

uint16_t f16_bits(double v) {
  const _Float16 h = (_Float16)v;
  uint16_t b;
  memcpy(&b, &h, 2);
  return b;
}
uint16_t bf16_bits(double v) {  // round to nearest even, via float
  const float f = (float)v;
  uint32_t u;
  memcpy(&u, &f, 4);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
double bf16_value(uint16_t b) {
  const uint32_t u = (uint32_t)b << 16;
  float f;
  memcpy(&f, &u, 4);
  return f;
}

// Natural pixel index (8 row + column) of element e of K-step s in lane
// half hh of the forward operand: rows 2s (e < 4) and 2s + 1, columns 4hh + e % 4.
int fwd_pixel(int s, int hh, int e) { return 8 * (2 * s + e / 4) + 4 * hh + e % 4; }
// Natural pixel index of output row i (0..63) of the inverse transform:
// i = 32 mt + 8 q + 4 hh + c is row 4 mt + q, column 4 hh + c.
int inv_pixel(int i) { return 8 * (4 * (i / 32) + (i % 32) / 8) + 4 * ((i % 8) / 4) + i % 4; }
// Zigzag position of element e of K-step s in lane half hh of the inverse
// operand: the forward output slot r = 8 (s % 2) + e of M-tile s / 2.
int inv_coef_z(int s, int hh, int e) { return 32 * (s / 2) + 8 * (2 * (s % 2) + e / 4) + 4 * hh + e % 4; }

}  // namespace

// Tables: f16 forward, f16 inverse, bf16 forward hi, bf16 forward lo, bf16
// inverse.  Layout: word ((mt * 4 + s) * 64 + lane) * 4 + w holds elements
// e = 2w, 2w+1 of lane `lane` for M-tile mt and K-step s, i.e. the A operand
// of v_mfma_f32_32x32x16: row i = 32 mt + lane % 32, columns
// k = 16 s + 8 (lane / 32) + e.  Forward tables: A[i][k] = B[n][p] for the
// coefficient at zigzag position i and pixel fwd_pixel(s, lane / 32, e);
// inverse tables: A[i][k] = B[n][p] for the coefficient at zigzag position
// inv_coef_z(s, lane / 32, e) and pixel inv_pixel(i).
void build_lp_tables(const double *basis, uint32_t (*lp)[kLpTableWords]) {
  static constexpr ZigZag zz{};
  for (int inv = 0; inv < 2; ++inv)
    for (int mt = 0; mt < 2; ++mt)
      for (int s = 0; s < 4; ++s)
        for (int l = 0; l < 64; ++l)
          for (int e = 0; e < 8; ++e) {
            const int i = 32 * mt + (l & 31), hh = l >> 5;
            const int n = inv ? zz.nat[inv_coef_z(s, hh, e)] : zz.nat[i];
            const int p = inv ? inv_pixel(i) : fwd_pixel(s, hh, e);
            const double v = basis[n * 64 + p];
            const uint16_t h16 = f16_bits(v);
            const uint16_t hb = bf16_bits(v);
            const uint16_t lb = bf16_bits(v - bf16_value(hb));
            const int word = ((mt * 4 + s) * 64 + l) * 4 + e / 2, sh = 16 * (e & 1);
            auto put = [&](int table, uint16_t bits) {
              if (sh == 0) lp[table][word] = 0u;
              lp[table][word] |= (uint32_t)bits << sh;
            };
            put(inv ? 1 : 0, h16);
            put(inv ? 4 : 2, hb);
            if (!inv) put(3, lb);
          }
}

namespace {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef _Float16 half2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// Streaming (non-temporal) 16- and 8-byte accesses: fragments and codes are
// touched once per call.
__device__ __forceinline__ uint4 nt_load16(const void *p) {
  const u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(p));
  return make_uint4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void nt_store16(void *p, const uint4 &v) {
  const u32x4 w = {v.x, v.y, v.z, v.w};
  __builtin_nontemporal_store(w, reinterpret_cast<u32x4 *>(p));
}
__device__ __forceinline__ uint2 nt_load8(const void *p) {
  const u32x2 v = __builtin_nontemporal_load(reinterpret_cast<const u32x2 *>(p));
  return make_uint2(v.x, v.y);
}
__device__ __forceinline__ void nt_store8(void *p, uint32_t a, uint32_t b) {
  const u32x2 w = {a, b};
  __builtin_nontemporal_store(w, reinterpret_cast<u32x2 *>(p));
}

// Tiles whose private bytes go through one AES pass together: a tile of
// DC + 9 AC holds 80 AES blocks, so two tiles fill three passes of 64 lanes
// where one tile alone takes two.
// Tiles whose private strings go through the cipher together: pairs in
// frag (DC + 9 AC: 160 AES blocks in 3 passes of 64 lanes), single tiles
// in defrag (80 blocks: one pass and a quad-lane pass for the last 16),
// which measured 2-4 us per 8192^2 image faster for defrag and slower for
// frag.  The fragment layout does not depend on the grouping.
constexpr uint32_t kFragGroup = 2, kDefragGroup = 1;

template <bool BF>
__device__ __forceinline__ f32x16 mfma(const uint4 &a, const uint4 &b, const f32x16 &c) {
  if constexpr (BF)
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0,
                                                   0, 0);
  else
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(half8, a), __builtin_bit_cast(half8, b), c, 0, 0,
                                                  0);
}

// Two FP32 values to two 16-bit storage values (round to nearest even), packed.
template <bool BF>
__device__ __forceinline__ uint32_t pack16(float a, float b) {
  const f32x2 v = {a, b};
  if constexpr (BF) return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
  else return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, half2v));
}

// A private integer (|q| <= 2040) as the operand pair (hi, lo): fp16 holds
// it exactly (lo = 0); bf16 keeps 8 significant bits in hi and the rest,
// exactly, in lo.
template <bool BF>
__device__ __forceinline__ void split_int(int32_t q, uint32_t &hi, uint32_t &lo) {
  if constexpr (BF) {
    const float f = (float)q;
    hi = (uint32_t)__builtin_bit_cast(uint16_t, (__bf16)f);
    lo = (uint32_t)__builtin_bit_cast(uint16_t, (__bf16)(f - __uint_as_float(hi << 16)));
  } else {
    hi = (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)(int16_t)q);
    lo = 0u;
  }
}

// Four pixel bytes (one row word) -> four exact 16-bit operand values in two
// words.  fp16: 0x6400 | x is 1024 + x, so one byte permute and one packed
// subtraction of 1024 give x.  bf16: the high half of the FP32 value.
template <bool BF>
__device__ __forceinline__ void pixels16(uint32_t w, uint32_t &lo, uint32_t &hi) {
  if constexpr (BF) {
    const uint32_t f0 = __float_as_uint((float)(w & 0xffu));
    const uint32_t f1 = __float_as_uint((float)((w >> 8) & 0xffu));
    const uint32_t f2 = __float_as_uint((float)((w >> 16) & 0xffu));
    const uint32_t f3 = __float_as_uint((float)(w >> 24));
    lo = __builtin_amdgcn_perm(f1, f0, 0x07060302u);
    hi = __builtin_amdgcn_perm(f3, f2, 0x07060302u);
  } else {
    const half2v k = {(_Float16)-1024.0f, (_Float16)-1024.0f};
    lo = __builtin_bit_cast(uint32_t, __builtin_bit_cast(half2v, __builtin_amdgcn_perm(0x64646464u, w, 0x04010400u)) + k);
    hi = __builtin_bit_cast(uint32_t, __builtin_bit_cast(half2v, __builtin_amdgcn_perm(0x64646464u, w, 0x04030402u)) + k);
  }
}

// Operand tables in LDS (copied once per workgroup): per table
// 2 x 4 x 64 lanes x 16 bytes.
// f16: forward, inverse; bf16: forward hi, forward lo, inverse.  The bf16
// forward keeps the basis to 16 significant bits (hi + lo) so the public
// coefficients meet their bound; the inverse only decides the residual
// codes, and one bf16 basis keeps those within +-1 (the residual absorbs the
// difference and both directions evaluate it identically).
template <bool BF>
struct LpLds {
  static constexpr int kFwd = 0, kFwdLo = 1, kInv = BF ? 2 : 1;
  uint4 t[BF ? 3 : 2][2 * 4 * 64];
};

template <bool BF>
__device__ __forceinline__ const uint4 &op(const LpLds<BF> &L, int table, int mt, int s, int lane) {
  return L.t[table][(mt * 4 + s) * 64 + lane];
}

template <bool BF>
__device__ __forceinline__ void load_lp_tables(LpLds<BF> &L, const uint32_t *tables, int tid, int nthreads) {
  const uint4 *src = reinterpret_cast<const uint4 *>(tables);
  constexpr int kWords4 = kLpTableWords / 4;  // uint4 per table
  for (int i = tid; i < kWords4; i += nthreads) {
    if constexpr (BF) {
      L.t[0][i] = src[2 * kWords4 + i];
      L.t[1][i] = src[3 * kWords4 + i];
      L.t[2][i] = src[4 * kWords4 + i];
    } else {
      L.t[0][i] = src[0 * kWords4 + i];
      L.t[1][i] = src[1 * kWords4 + i];
    }
  }
}

// One lane's B operand of the int8 quantiser for one pass of up to 16
// private coefficients (v_mfma_i32_16x16x64_i8, A = 16 blocks x 64 samples):
// column lane % 16 (private rank 16 pass + lane % 16), samples 16 g .. 16 g + 15
// (g = lane / 16) in the order of the A operand built by lp_quant_operands:
// dword r covers row 4 (g / 2) + r, columns 4 (g % 2) .. + 3, i.e. word
// 2 (4 (g / 2) + r) + g % 2 of the natural-order limb rows.  Limbs low, mid,
// high; bias = 128 sum_p Bq split as beta2 2^16 + beta1 2^8 + beta0.
struct LpQ2 {
  q2v4 limb[3];
  int32_t beta[3];
  int32_t pad;
};

__device__ __forceinline__ LpQ2 lp_q2_operand(const uint32_t *q2, int n, int lane) {
  LpQ2 o;
  const int g = lane >> 4;
#pragma unroll
  for (int L = 0; L < 3; ++L)
#pragma unroll
    for (int r = 0; r < 4; ++r)
      o.limb[L][r] = n >= 0 ? (int)q2[n * kQ2RowWords + 16 * L + 2 * (4 * (g >> 1) + r) + (g & 1)] : 0;
  const int32_t bias = n >= 0 ? (int32_t)q2[n * kQ2RowWords + 48] : 0;
  o.beta[0] = bias & 0xff;
  o.beta[1] = (bias >> 8) & 0xff;
  o.beta[2] = bias >> 16;
  o.pad = 0;
  return o;
}

// The int8 A operands of one half (16 blocks each: blocks 0-15 and 16-31 of
// the half): lane row R = lane / 16 of the pixel words holds, for block
// lane % 16 of group R % 2, the columns 4 (R / 2) .. + 3 of rows 0-7 (lo:
// rows 0-3, hi: rows 4-7).  A 32-lane swap of lo with hi, then a 16-lane
// swap, leaves in lo (group 0) and hi (group 1) the layout lane row g:
// rows 4 (g / 2) .. + 3, columns 4 (g % 2) .. + 3 of block lane % 16.
__device__ __forceinline__ void lp_quant_operands(const uint32_t (&xr)[8], q2v4 &a0, q2v4 &a1) {
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const auto s32 = __builtin_amdgcn_permlane32_swap(xr[r] ^ 0x80808080u, xr[4 + r] ^ 0x80808080u, false, false);
    const auto s16 = __builtin_amdgcn_permlane16_swap(s32[0], s32[1], false, false);
    a0[r] = (int)s16[0];
    a1[r] = (int)s16[1];
  }
}

// Private integers of one 16-block group: D row 4 (lane / 16) + r (block),
// column lane % 16 (private rank), exact as the plain form's q2_acc.
__device__ __forceinline__ q2v4 lp_quant(const q2v4 &a, const LpQ2 &Q) {
  q2v4 c = {Q.beta[2], Q.beta[2], Q.beta[2], Q.beta[2]};
  c = __builtin_amdgcn_mfma_i32_16x16x64_i8(a, Q.limb[2], c, 0, 0, 0);
  c = (q2v4)(((q2u4)c << 8u) + (q2u4)Q.beta[1]);
  c = __builtin_amdgcn_mfma_i32_16x16x64_i8(a, Q.limb[1], c, 0, 0, 0);
  c = (q2v4)(((q2u4)c << 8u) + (q2u4)Q.beta[0]);
  c = __builtin_amdgcn_mfma_i32_16x16x64_i8(a, Q.limb[0], c, 0, 0, 0);
#pragma unroll
  for (int r = 0; r < 4; ++r) c[r] = q2_round(c[r]);
  return c;
}

// Coefficient bookkeeping of zigzag position z: compile-time for "DC + k AC"
// selections, wave-uniform otherwise.  rank = rank among the private
// (private) or the public positions.
struct ZSlot {
  uint32_t priv;
  uint32_t rank;
};
template <class MP>
__device__ __forceinline__ ZSlot zslot(uint64_t mask, int z) {
  ZSlot c;
  if constexpr (MP::kStatic) {
    c.priv = z < MP::kNPriv ? 1u : 0u;
    c.rank = c.priv ? (uint32_t)z : (uint32_t)(z - MP::kNPriv);
  } else {
    const uint32_t before = (uint32_t)__builtin_popcountll(mask & ((1ull << z) - 1ull));
    c.priv = (uint32_t)((mask >> z) & 1u);
    c.rank = c.priv ? before : (uint32_t)z - before;
  }
  return c;
}

struct LpArgs {
  TileGeom g;
  uint16_t *pub;        // frag: out; defrag: in
  uint8_t *priv;        // frag: out; defrag: in
  uint8_t *resid;       // 16-byte code record per block
  uint8_t *pix_out;     // defrag
  ExcSlots exc;
  uint32_t *status;
  const uint32_t *q2;
  const uint32_t *tables;  // kLpTables x kLpTableWords
  const uint32_t *aes_t0;
  AesArgs aes;
  uint32_t npass;          // int8 quantiser passes, ceil(npriv / 16)
  uint32_t pstride;        // LDS bytes of one tile's private stage
  uint32_t wave_lds;       // LDS bytes per wave
  uint32_t plist[16];      // natural indices of the private positions, 4 per word
};

// LDS of one wave: one private stage per tile of its group (int16
// [rank][block], the tile's private byte string), then (frag) the public
// stage of one half (npub rows of 64 bytes: 32 blocks of a rank).
struct WaveLds {
  uint8_t *priv;
  uint8_t *pub;
};

// The tile's private byte string is AES-CTR encrypted (frag) or decrypted
// (defrag) for the tiles of a group at once: lane i of a pass takes AES
// block a = 64 pass + i of the concatenated tiles.  Tile t's bytes start at
// byte 128 P t of the fragment, i.e. counter 8 P t.
struct TileGroup {
  uint32_t n;         // tiles in the group (1 or 2)
  uint32_t t0, t1;    // the tiles
  uint32_t nb0, nb1;  // blocks in each tile
};

// AES blocks a = first + lane / 4 of the group, one per quad of lanes
// (aes_encrypt_quad), 4 bytes per lane.  Called by the whole wave, with the
// cipher on.
template <bool kEncrypt, int LPB = 4>
__device__ __forceinline__ void group_ctr_tail(const TileGroup &G, const WaveLds &W, uint32_t pstride, uint8_t *gpriv,
                                               uint32_t npriv, int lane, const AesLds &s_aes, const AesArgs &aes,
                                               uint32_t first, uint32_t n0, uint32_t total) {
  constexpr uint32_t WB = 16u / LPB;
  (void)lane;
  const uint32_t ln = fresh_lane();
  const uint32_t a = first + ln / LPB, part = ln % LPB;
  const bool live = a < total;
  const bool second = a >= n0;
  const uint32_t i = second ? a - n0 : a;
  const uint32_t t = second ? G.t1 : G.t0;
  const uint32_t tbytes = 2u * npriv * (second ? G.nb1 : G.nb0);
  const uint32_t o = 16u * i + WB * part;
  uint8_t *lp = W.priv + (second ? pstride : 0u) + o;
  uint8_t *gp = gpriv + (uint64_t)t * 128u * npriv + o;
  uint32_t v[WB / 4];
#pragma unroll
  for (uint32_t k = 0; k < WB / 4; ++k) v[k] = 0u;
  if (live) {
    if (kEncrypt || o + WB <= tbytes) {
      const uint8_t *src = kEncrypt ? (const uint8_t *)lp : (const uint8_t *)gp;
#pragma unroll
      for (uint32_t k = 0; k < WB / 4; ++k) v[k] = reinterpret_cast<const uint32_t *>(src)[k];
    } else {  // the fragment's final, partial AES block: never read past its end
      for (uint32_t j = 0; j + o < tbytes; ++j) v[j >> 2] |= (uint32_t)gp[j] << (8u * (j & 3u));
    }
  }
  uint32_t w[4];
  aes_counter(aes.ctr_hi, aes.ctr_lo, (uint64_t)t * 8u * npriv + i, w[0], w[1], w[2], w[3]);
  static_assert(LPB == 4, "one block per quad of lanes");
  v[0] ^= aes_encrypt_quad(part == 0 ? w[0] : part == 1 ? w[1] : part == 2 ? w[2] : w[3], part, s_aes);
  if (live) {
    if (!kEncrypt || o + WB <= tbytes) {
      uint8_t *dst = kEncrypt ? gp : lp;
#pragma unroll
      for (uint32_t k = 0; k < WB / 4; ++k) reinterpret_cast<uint32_t *>(dst)[k] = v[k];
    } else {
      for (uint32_t j = 0; j + o < tbytes; ++j) gp[j] = (uint8_t)(v[j >> 2] >> (8u * (j & 3u)));
    }
  }
}

// Whole passes of 64 AES blocks take one block per lane; a last pass of at
// most 16 blocks takes one block per quad of lanes.
template <bool kEncrypt>
__device__ __forceinline__ void group_ctr(const TileGroup &G, const WaveLds &W, uint32_t pstride, uint8_t *gpriv,
                                          uint32_t npriv, int lane, const AesLds &s_aes, const AesArgs &aes) {
  const uint32_t n0 = (2u * npriv * G.nb0 + 15u) / 16u;
  const uint32_t total = n0 + (G.n > 1 ? (2u * npriv * G.nb1 + 15u) / 16u : 0u);
  const uint32_t rem = total & 63u;
  const uint32_t nrow = aes.enabled && rem != 0u && rem <= 16u ? total - rem : total;  // wave-uniform
  for (uint32_t a = (uint32_t)lane; a < nrow; a += 64u) {
    const bool second = a >= n0;
    const uint32_t i = second ? a - n0 : a;
    const uint32_t t = second ? G.t1 : G.t0;
    const uint32_t tbytes = 2u * npriv * (second ? G.nb1 : G.nb0);
    uint8_t *lp = W.priv + (second ? pstride : 0u) + 16u * i;
    uint8_t *gp = gpriv + (uint64_t)t * 128u * npriv + 16u * i;
    uint4 v;
    if (kEncrypt) {
      v = *reinterpret_cast<const uint4 *>(lp);
    } else if (16u * i + 16u <= tbytes) {
      v = nt_load16(gp);
    } else {  // the fragment's final, partial AES block: never read past its end
      uint32_t w[4] = {0u, 0u, 0u, 0u};
      for (uint32_t j = 0; j < tbytes - 16u * i; ++j) w[j >> 2] |= (uint32_t)gp[j] << (8u * (j & 3u));
      v = make_uint4(w[0], w[1], w[2], w[3]);
    }
    if (aes.enabled) {
      uint32_t w0, w1, w2, w3;
      aes_counter(aes.ctr_hi, aes.ctr_lo, (uint64_t)t * 8u * npriv + i, w0, w1, w2, w3);
      aes_encrypt(w0, w1, w2, w3, s_aes);
      v.x ^= w0;
      v.y ^= w1;
      v.z ^= w2;
      v.w ^= w3;
    }
    if (!kEncrypt) {
      *reinterpret_cast<uint4 *>(lp) = v;
    } else if (16u * i + 16u <= tbytes) {
      nt_store16(gp, v);
    } else {
      const uint32_t w[4] = {v.x, v.y, v.z, v.w};
      for (uint32_t j = 0; j < tbytes - 16u * i; ++j) gp[j] = (uint8_t)(w[j >> 2] >> (8u * (j & 3u)));
    }
  }
  if (nrow != total) group_ctr_tail<kEncrypt>(G, W, pstride, gpriv, npriv, lane, s_aes, aes, nrow, n0, total);
}

// The eight row words (columns 4h .. 4h + 3) of the lane's block in one half;
// img spans the whole image (fewer than 2^32 samples), rows are W apart.
__device__ __forceinline__ void load_rows(const TileGeom &g, __amdgpu_buffer_rsrc_t img, uint32_t t, uint32_t nt,
                                          int lane, uint32_t (&xr)[8]) {
  const uint64_t b = (uint64_t)t * 64u + 32u * nt + ((uint32_t)lane & 31u);
  const bool valid = b < g.nb;
  const uint32_t voff = valid ? block_origin(g, (uint32_t)b) + 4u * (fresh_lane() >> 5) : 0u;
#pragma unroll
  for (int r = 0; r < 8; ++r)
    xr[r] = valid ? __builtin_amdgcn_raw_buffer_load_b32(img, voff, (int)(r * g.W), kNonTemporal) : 0u;
}

// The one reconstruction routine: y[mt] (rows 4 mt .. 4 mt + 3 of the lane's
// block, columns 4h .. 4h + 3; element 4 q + c is row 4 mt + q, column
// 4h + c) from the operands chi (and, for bf16, clo: the low halves of the
// private integers, nonzero only in K-steps that hold private positions).
template <bool BF>
__device__ __forceinline__ void lp_idct(const LpLds<BF> &L, int lane, const uint4 (&chi)[4], const uint4 (&clo)[4],
                                        const bool (&has_lo)[4], f32x16 (&y)[2]) {
#pragma unroll
  for (int mt = 0; mt < 2; ++mt) {
    f32x16 acc = {};
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      acc = mfma<BF>(op(L, LpLds<BF>::kInv, mt, s, lane), chi[s], acc);
      if constexpr (BF)
        if (has_lo[s]) acc = mfma<BF>(op(L, LpLds<BF>::kInv, mt, s, lane), clo[s], acc);
    }
    y[mt] = acc;
  }
}

// Four reconstructed samples of row word 4 q4 .. 4 q4 + 3 of y, rounded half
// to even and clamped to [0, 255] (v_cvt_pk_u8_f32), one per byte.
__device__ __forceinline__ uint32_t rec_word(const f32x16 &y, int q4) {
  uint32_t w = 0u;
#pragma unroll
  for (int e = 0; e < 4; ++e) w = __builtin_amdgcn_cvt_pk_u8_f32(y[4 * q4 + e], e, w);
  return w;
}

// Residual codes of one row word: per byte (x - rec) mod 4, i.e. 0, 1 (+1),
// 3 (-1) for |x - rec| <= 1, without borrows between bytes.
__device__ __forceinline__ uint32_t row_codes(uint32_t x, uint32_t rec) {
  return (((x & 0x03030303u) | 0x04040404u) - (rec & 0x03030303u)) & 0x03030303u;
}

// Applies the codes of row word m (bits 0-1 of each byte) to rec: +1 for
// code 1, -1 for code 3, nothing for 0 and 2 (2: the exception slots hold the
// sample).  The result is the sample, in [0, 255], so no byte carries.
__device__ __forceinline__ uint32_t apply_codes(uint32_t rec, uint32_t m) {
  const uint32_t m1 = m >> 1;
  return rec + (m & ~m1 & 0x01010101u) - (m & m1 & 0x01010101u);
}

template <class MP>
__device__ __forceinline__ uint64_t mask_of(const TileGeom &g) {
  return MP::kStatic ? g.mask : opaque_u64(g.mask);
}

// The lane's coefficient of the slot pair at zigzag positions z0 (lane half
// 0) and z0 + 4 (lane half 1), with the stage and fragment offsets of its
// value.  Private integers sit in the stage as int16 [rank][64 blocks];
// public values of a half in the public stage as [rank][32 blocks].  For
// "DC + k AC" selections two private (or two public) positions of a pair
// are 4 ranks apart, so the offsets are a per-lane base plus a constant.
template <class MP>
struct Pair {
  ZSlot c0, c1;
  bool any_priv, both_priv, any_pub, both_pub;
  bool mine_priv;
  __device__ __forceinline__ Pair(uint64_t mask, int z0, uint32_t h) {
    c0 = zslot<MP>(mask, z0);
    c1 = zslot<MP>(mask, z0 + 4);
    any_priv = (c0.priv | c1.priv) != 0u;
    both_priv = (c0.priv & c1.priv) != 0u;
    any_pub = !both_priv;
    both_pub = !any_priv;
    mine_priv = h ? c1.priv != 0u : c0.priv != 0u;
  }
  // stage byte offset of the private integer this lane reads (for a pair with
  // one private half, that half's integer, read by every lane)
  __device__ __forceinline__ uint32_t priv_off(uint32_t jb, uint32_t h) const {
    if constexpr (MP::kStatic) {
      return both_priv ? 128u * c0.rank + (2u * jb + 512u * h) : 128u * (c0.priv ? c0.rank : c1.rank) + 2u * jb;
    } else {
      const uint32_t r = both_priv ? (h ? c1.rank : c0.rank) : (c0.priv ? c0.rank : c1.rank);
      return 128u * r + 2u * jb;
    }
  }
  // public rank this lane stores or loads (for a pair with one public half,
  // that half's rank)
  __device__ __forceinline__ uint32_t pub_rank(uint32_t h) const {
    return both_pub ? (h ? c1.rank : c0.rank) : (c0.priv ? c1.rank : c0.rank);
  }
};

// Moves the private integers of a partial tile (ntb < 64 blocks) between
// the stage layout [rank][64] and the fragment's [rank][ntb] (pack: before
// encryption; unpack: after decryption), in place, one rank at a time in the
// order that never overwrites a value still to be moved.
template <bool kPack>
__device__ __forceinline__ void stage_repack(uint8_t *stage, uint32_t npriv, uint32_t ntb, int) {
  const uint32_t lane = fresh_lane();
  for (uint32_t k = 1; k < npriv; ++k) {
    const uint32_t r = kPack ? k : npriv - k;
    const bool mine = lane < ntb;
    const uint32_t from = kPack ? 128u * r : 2u * r * ntb, to = kPack ? 2u * r * ntb : 128u * r;
    const int16_t v = mine ? *reinterpret_cast<const int16_t *>(stage + from + 2u * lane) : (int16_t)0;
    wave_lds_sync();
    if (mine) *reinterpret_cast<int16_t *>(stage + to + 2u * lane) = v;
    wave_lds_sync();
  }
}

// ---------------------------------------------------------------------------
// frag
// Register budget: 4 waves per SIMD (128 VGPRs) for both storage types
// (bf16 frag spills 2 registers there and still runs 7-8 % faster than at
// 3 waves per SIMD with 138 VGPRs).
template <bool BF>
constexpr int lp_waves_per_eu() {
  return 4;
}

template <bool BF, class MP>
__global__ __launch_bounds__(512, lp_waves_per_eu<BF>()) void lp_frag_kernel(LpArgs a) {
  __shared__ AesLds s_aes;
  __shared__ LpLds<BF> s_tab;
  extern __shared__ __attribute__((aligned(16))) uint8_t s_dyn[];
  const int lane = threadIdx.x & 63;
  const uint32_t nw = blockDim.x >> 6;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const TileGeom &g = a.g;
  LpQ2 *s_q2 = reinterpret_cast<LpQ2 *>(s_dyn);
  if (a.aes.enabled) aes_load_tables(s_aes, a.aes_t0, a.aes.key, threadIdx.x, blockDim.x);
  load_lp_tables<BF>(s_tab, a.tables, threadIdx.x, blockDim.x);
  for (uint32_t i = threadIdx.x; i < 64u * a.npass; i += blockDim.x) {
    const uint32_t rank = 16u * (i >> 6) + (i & 15u);
    const int n = rank < g.npriv ? (int)((a.plist[rank >> 2] >> (8u * (rank & 3u))) & 0xffu) : -1;
    s_q2[i] = lp_q2_operand(a.q2, n, (int)(i & 63u));
  }
  __syncthreads();
  WaveLds W;
  W.priv = s_dyn + 64u * a.npass * sizeof(LpQ2) + wave * a.wave_lds;
  W.pub = W.priv + kFragGroup * a.pstride;
  const uint64_t mask = mask_of<MP>(g);
  const uint32_t h = (uint32_t)lane >> 5, jl = (uint32_t)lane & 31u;
  const uint32_t stride = gridDim.x * nw;
  const uint32_t npriv = g.npriv, npub = g.npub;
  const __amdgpu_buffer_rsrc_t img = buffer_rsrc(g.pix, (uint32_t)(g.nb * 64u));
  const __amdgpu_buffer_rsrc_t res = buffer_rsrc(a.resid, (uint32_t)(g.nb * 16u));

  uint32_t t = blockIdx.x * nw + wave;
  uint32_t xn[8];  // the next half's pixel rows, in flight during the current half
  if (t < g.ntiles) load_rows(g, img, t, 0, lane, xn);
  while (t < g.ntiles) {
    TileGroup G;
    G.n = 0;
    for (uint32_t gi = 0; gi < kFragGroup && t < g.ntiles; ++gi, t += stride) {
      const uint64_t b0 = (uint64_t)t * 64u;
      const uint32_t ntb = (uint32_t)min<uint64_t>(64u, g.nb - b0);
      if (gi == 0) {
        G.t0 = t;
        G.nb0 = ntb;
      } else {
        G.t1 = t;
        G.nb1 = ntb;
      }
      G.n = gi + 1;
      uint8_t *stage = W.priv + gi * a.pstride;
      const uint32_t tn = t + stride;
      uint32_t tile_exc = 0;  // wave-uniform
#pragma unroll 1
      for (uint32_t nt = 0; nt < 2; ++nt) {
        const uint32_t jb = 32u * nt + jl;
        const bool bv = jb < ntb;
        uint32_t xr[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) xr[r] = xn[r];
        if (nt == 0) load_rows(g, img, t, 1, lane, xn);
        else if (tn < g.ntiles) load_rows(g, img, tn, 0, lane, xn);

        // ---- private integers (int8 matrix products), into the stage
        {
          q2v4 a0, a1;
          lp_quant_operands(xr, a0, a1);
          for (uint32_t p = 0; p < a.npass; ++p) {
            const LpQ2 Q = s_q2[64u * p + lane];
            const uint32_t rank = 16u * p + (uint32_t)(lane & 15);
#pragma unroll
            for (int grp = 0; grp < 2; ++grp) {
              const q2v4 q = lp_quant(grp ? a1 : a0, Q);
              const uint32_t blk = 32u * nt + 16u * grp + 4u * ((uint32_t)lane >> 4);
              if (rank < npriv)
                *reinterpret_cast<uint2 *>(stage + 128u * rank + 2u * blk) =
                    make_uint2(__builtin_amdgcn_perm((uint32_t)q[1], (uint32_t)q[0], 0x05040100u),
                               __builtin_amdgcn_perm((uint32_t)q[3], (uint32_t)q[2], 0x05040100u));
            }
          }
        }

        // ---- forward transform: C^T = K X^T, M = coefficient (zigzag), N = block
        f32x16 acc[2];
        {
          uint4 bx[4];
#pragma unroll
          for (int s = 0; s < 4; ++s) {
            uint32_t w0, w1, w2, w3;
            pixels16<BF>(xr[2 * s], w0, w1);
            pixels16<BF>(xr[2 * s + 1], w2, w3);
            bx[s] = make_uint4(w0, w1, w2, w3);
          }
#pragma unroll
          for (int mt = 0; mt < 2; ++mt) {
            f32x16 c = {};
#pragma unroll
            for (int s = 0; s < 4; ++s) {
              c = mfma<BF>(op(s_tab, LpLds<BF>::kFwd, mt, s, lane), bx[s], c);
              if constexpr (BF) c = mfma<BF>(op(s_tab, LpLds<BF>::kFwdLo, mt, s, lane), bx[s], c);
            }
            acc[mt] = c;
          }
        }
        wave_lds_sync();  // the stage's private integers, written above by other lanes

        // ---- stored values: public ones to the half's stage rows and the
        // inverse operands; private ones are the integers
        uint4 chi[4], clo[4];
        bool has_lo[4];
        static_for<0, 4>([&](auto sc) {
          constexpr int s = decltype(sc)::value, mt = s / 2, sg = s % 2;
          uint32_t hw[4], lw[4];
          bool any_lo = false;
          static_for<0, 4>([&](auto pc) {
            constexpr int pr = decltype(pc)::value;
            constexpr int r0 = 8 * sg + 2 * pr;  // slots r0, r0 + 1 of M-tile mt
            uint32_t w = pack16<BF>(acc[mt][r0], acc[mt][r0 + 1]);
            uint32_t lo = 0u;
            static_for<0, 2>([&](auto ec) {
              constexpr int e = decltype(ec)::value, r = r0 + e;
              const Pair<MP> P(mask, 32 * mt + 8 * (r / 4) + (r % 4), h);
              if (P.any_priv) {
                const int32_t q = (int32_t) * reinterpret_cast<const int16_t *>(stage + P.priv_off(jb, h));
                uint32_t qh, ql;
                split_int<BF>(q, qh, ql);
                if (P.mine_priv) {
                  w = e ? ((w & 0x0000ffffu) | (qh << 16)) : ((w & 0xffff0000u) | qh);
                  lo |= ql << (16 * e);
                }
                any_lo = true;
              }
              if (P.any_pub && !P.mine_priv) {
                const uint16_t v = bv ? (uint16_t)(e ? (w >> 16) : w) : (uint16_t)0;
                if constexpr (MP::kStatic)
                  *reinterpret_cast<uint16_t *>(W.pub + (P.both_pub ? 64u * P.c0.rank + (2u * jl + 256u * h)
                                                                    : 64u * P.c1.rank + 2u * jl)) = v;
                else
                  *reinterpret_cast<uint16_t *>(W.pub + 64u * P.pub_rank(h) + 2u * jl) = v;
              }
            });
            hw[pr] = w;
            lw[pr] = lo;
          });
          chi[s] = make_uint4(hw[0], hw[1], hw[2], hw[3]);
          clo[s] = make_uint4(lw[0], lw[1], lw[2], lw[3]);
          has_lo[s] = BF && any_lo;
        });

        // ---- reconstruction and residual codes
        f32x16 y[2];
        lp_idct<BF>(s_tab, lane, chi, clo, has_lo, y);
        uint32_t rec[8];
        uint32_t sad = 0u;
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          rec[r] = rec_word(y[r / 4], r % 4);
          sad = __builtin_amdgcn_sad_u8(xr[r], rec[r], sad);
        }
        uint32_t code[2] = {0u, 0u};
        if (__builtin_amdgcn_ballot_w64(sad != 0u) != 0ull) {
          uint32_t m[8], odd = 0u;
#pragma unroll
          for (int r = 0; r < 8; ++r) {
            m[r] = row_codes(xr[r], rec[r]);
            odd += (uint32_t)__builtin_popcount(m[r] & 0x01010101u);
          }
          // a sample with |r| >= 2 adds at least 2 to sad and at most 1 to odd
          if (__builtin_amdgcn_ballot_w64(sad > odd && bv) != 0ull) {
            uint32_t nesc = 0;
#pragma unroll
            for (int r = 0; r < 8; ++r)
#pragma unroll
              for (int c = 0; c < 4; ++c) {
                const int d = (int)((xr[r] >> (8 * c)) & 0xffu) - (int)((rec[r] >> (8 * c)) & 0xffu);
                nesc += (bv && (d > 1 || d < -1)) ? 1u : 0u;
              }
            uint32_t total;
            uint32_t slot = tile_exc + wave_exclusive_scan(nesc, lane, total);
#pragma unroll
            for (int r = 0; r < 8; ++r)
#pragma unroll
              for (int c = 0; c < 4; ++c) {
                const uint32_t xv = (xr[r] >> (8 * c)) & 0xffu;
                const int d = (int)xv - (int)((rec[r] >> (8 * c)) & 0xffu);
                if (bv && (d > 1 || d < -1)) {
                  m[r] = (m[r] & ~(3u << (8 * c))) | (2u << (8 * c));
                  if (slot < a.exc.per_tile) {
                    a.exc.pos[(size_t)t * a.exc.per_tile + slot] = (uint16_t)(jb * 64u + 8u * r + 4u * h + c);
                    a.exc.val[(size_t)t * a.exc.per_tile + slot] = (uint8_t)xv;
                  }
                  ++slot;
                }
              }
            tile_exc += total;
          }
#pragma unroll
          for (int r = 0; r < 8; ++r) code[r / 4] |= m[r] << (2 * (r % 4));
        }
        if (bv) {
          const uint32_t off = 16u * (uint32_t)(b0 + jb) + 8u * h;
          const u32x2 cw = {code[0], code[1]};  // one 8-byte store: a half writes 512 contiguous bytes
          __builtin_amdgcn_raw_buffer_store_b64(cw, res, off, 0, kNonTemporal);
        }

        // ---- this half's public values: the half's region of the fragment
        // ([rank][32 blocks], contiguous) leaves as 16-byte stores, whole
        // cache lines per instruction
        wave_lds_sync();
        uint16_t *pub_tile = a.pub + b0 * npub;
        if (ntb == 64u) {
          const __amdgpu_buffer_rsrc_t prs = buffer_rsrc(pub_tile, npub * 128u);
          for (uint32_t c = (uint32_t)lane; c < 4u * npub; c += 64u) {
            const uint4 v = *reinterpret_cast<const uint4 *>(W.pub + 16u * c);
            const u32x4 vv = {v.x, v.y, v.z, v.w};
            __builtin_amdgcn_raw_buffer_store_b128(vv, prs, 64u * npub * nt + 16u * c, 0, kNonTemporal);
          }
        } else {
          const uint32_t m0 = min(32u, ntb), nv = ntb > 32u * nt ? min(32u, ntb - 32u * nt) : 0u;
          for (uint32_t c = (uint32_t)lane; c < 32u * npub; c += 64u) {
            const uint32_t r = c >> 5, j = c & 31u;
            if (j < nv)
              pub_tile[nt * npub * m0 + r * nv + j] = *reinterpret_cast<const uint16_t *>(W.pub + 64u * r + 2u * j);
          }
        }
        wave_lds_sync();
      }
      if (lane == 0) a.exc.count[t] = (uint16_t)min(tile_exc, 0xffffu);
      if (tile_exc > a.exc.per_tile && lane == 0 && a.status) atomicOr(a.status, SF_STATUS_EXC_OVERFLOW);
      if (ntb < 64u) stage_repack<true>(stage, npriv, ntb, lane);
    }
    // ---- the group's private bytes: AES-CTR and coalesced stores
    group_ctr<true>(G, W, a.pstride, a.priv, npriv, lane, s_aes, a.aes);
    wave_lds_sync();
  }
}

// ---------------------------------------------------------------------------
// defrag
template <bool BF, class MP>
__global__ __launch_bounds__(512, lp_waves_per_eu<BF>()) void lp_defrag_kernel(LpArgs a) {
  __shared__ AesLds s_aes;
  __shared__ LpLds<BF> s_tab;
  extern __shared__ __attribute__((aligned(16))) uint8_t s_dyn[];
  const int lane = threadIdx.x & 63;
  const uint32_t nw = blockDim.x >> 6;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const TileGeom &g = a.g;
  if (a.aes.enabled) aes_load_tables(s_aes, a.aes_t0, a.aes.key, threadIdx.x, blockDim.x);
  load_lp_tables<BF>(s_tab, a.tables, threadIdx.x, blockDim.x);
  __syncthreads();
  WaveLds W;
  W.priv = s_dyn + wave * a.wave_lds;
  W.pub = nullptr;
  const uint64_t mask = mask_of<MP>(g);
  const uint32_t h = (uint32_t)lane >> 5, jl = (uint32_t)lane & 31u;
  const uint32_t stride = gridDim.x * nw;
  const uint32_t npub = g.npub;
  const __amdgpu_buffer_rsrc_t img = buffer_rsrc(a.pix_out, (uint32_t)(g.nb * 64u));
  const __amdgpu_buffer_rsrc_t res = buffer_rsrc(a.resid, (uint32_t)(g.nb * 16u));

  for (uint32_t t0 = blockIdx.x * nw + wave; t0 < g.ntiles;) {
    TileGroup G;
    G.t0 = t0;
    G.nb0 = (uint32_t)min<uint64_t>(64u, g.nb - (uint64_t)t0 * 64u);
    G.t1 = t0 + stride;
    G.n = kDefragGroup > 1 && G.t1 < g.ntiles ? 2u : 1u;
    G.nb1 = G.n > 1 ? (uint32_t)min<uint64_t>(64u, g.nb - (uint64_t)G.t1 * 64u) : 0u;
    t0 += G.n * stride;
    group_ctr<false>(G, W, a.pstride, a.priv, g.npriv, lane, s_aes, a.aes);
    wave_lds_sync();
    for (uint32_t gi = 0; gi < G.n; ++gi) {
      const uint32_t t = gi ? G.t1 : G.t0, ntb = gi ? G.nb1 : G.nb0;
      const uint64_t b0 = (uint64_t)t * 64u;
      uint8_t *stage = W.priv + gi * a.pstride;
      if (ntb < 64u) stage_repack<false>(stage, g.npriv, ntb, lane);
      const __amdgpu_buffer_rsrc_t prs = buffer_rsrc(a.pub + b0 * npub, npub * ntb * 2u);
      const uint32_t nexc = (uint32_t)__builtin_amdgcn_readfirstlane(a.exc.count[t]);
#pragma unroll 1
      for (uint32_t nt = 0; nt < 2; ++nt) {
        const uint32_t jb = 32u * nt + jl;
        const bool bv = jb < ntb;
        const uint32_t roff = 16u * (uint32_t)(b0 + jb) + 8u * h;
        uint32_t code0 = 0u, code1 = 0u;
        if (bv) {
          const u32x2 cw = __builtin_amdgcn_raw_buffer_load_b64(res, roff, 0, kNonTemporal);
          code0 = cw.x;
          code1 = cw.y;
        }
        // ---- operands: public values straight from the fragment (half-
        // relative offsets: the half's region holds [rank][m blocks], and the
        // pair's ranks are 4 apart for "DC + k AC"), private integers from
        // the decrypted stage
        const uint32_t m0 = min(32u, ntb), mh = nt ? (ntb > 32u ? ntb - 32u : 0u) : m0;
        const uint32_t vbase = 2u * (nt * npub * m0 + jl), vbase4 = vbase + 8u * mh * h;
        uint4 chi[4], clo[4];
        bool has_lo[4];
        static_for<0, 4>([&](auto sc) {
          constexpr int s = decltype(sc)::value, mt = s / 2, sg = s % 2;
          uint32_t hw[4], lw[4];
          bool any_lo = false;
          static_for<0, 4>([&](auto pc) {
            constexpr int pr = decltype(pc)::value;
            constexpr int r0 = 8 * sg + 2 * pr;
            uint32_t w = 0u, lo = 0u;
            static_for<0, 2>([&](auto ec) {
              constexpr int e = decltype(ec)::value, r = r0 + e;
              const Pair<MP> P(mask, 32 * mt + 8 * (r / 4) + (r % 4), h);
              uint32_t v = 0u;
              if (P.any_priv) {
                const int32_t q = (int32_t) * reinterpret_cast<const int16_t *>(stage + P.priv_off(jb, h));
                uint32_t qh, ql;
                split_int<BF>(q, qh, ql);
                if (P.mine_priv) {
                  v = qh;
                  lo |= ql << (16 * e);
                }
                any_lo = true;
              }
              if (P.any_pub) {
                uint32_t pv;
                if constexpr (MP::kStatic)
                  pv = P.both_pub ? __builtin_amdgcn_raw_buffer_load_b16(prs, vbase4, (int)(2u * mh * P.c0.rank), 0)
                                  : __builtin_amdgcn_raw_buffer_load_b16(prs, vbase, (int)(2u * mh * P.c1.rank), 0);
                else
                  pv = __builtin_amdgcn_raw_buffer_load_b16(prs, vbase + 2u * mh * P.pub_rank(h), 0, 0);
                if (!P.mine_priv) v = pv;
              }
              w |= v << (16 * e);
            });
            hw[pr] = w;
            lw[pr] = lo;
          });
          chi[s] = make_uint4(hw[0], hw[1], hw[2], hw[3]);
          clo[s] = make_uint4(lw[0], lw[1], lw[2], lw[3]);
          has_lo[s] = BF && any_lo;
        });
        f32x16 y[2];
        lp_idct<BF>(s_tab, lane, chi, clo, has_lo, y);
        uint32_t out[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) out[r] = rec_word(y[r / 4], r % 4);
        if (__builtin_amdgcn_ballot_w64((code0 | code1) != 0u) != 0ull) {
#pragma unroll
          for (int r = 0; r < 8; ++r) out[r] = apply_codes(out[r], ((r < 4 ? code0 : code1) >> (2 * (r % 4))) & 0x03030303u);
        }
        // samples kept in the exception slots (code 2), patched by the lane that owns them
        for (uint32_t e = 0; e < min(nexc, a.exc.per_tile); ++e) {
          const uint32_t pos = a.exc.pos[(size_t)t * a.exc.per_tile + e];
          const uint32_t val = a.exc.val[(size_t)t * a.exc.per_tile + e];
          const uint32_t p = pos & 63u;
          if ((pos >> 6) == jb && ((p >> 2) & 1u) == h) {
            const uint32_t r = p >> 3, c = p & 3u;
#pragma unroll
            for (int rr = 0; rr < 8; ++rr)
              if ((uint32_t)rr == r) out[rr] = (out[rr] & ~(0xffu << (8u * c))) | (val << (8u * c));
          }
        }
        if (bv) {
          const uint32_t voff = block_origin(g, (uint32_t)(b0 + jb)) + 4u * h;
#pragma unroll
          for (int r = 0; r < 8; ++r) __builtin_amdgcn_raw_buffer_store_b32(out[r], img, voff, (int)(r * g.W), kNonTemporal);
        }
      }
    }
    wave_lds_sync();
  }
}

// ---------------------------------------------------------------------------
// launchers
// Dynamic LDS of a workgroup: `shared` (frag: the quantiser's B operands)
// plus `per_wave` for each wavefront (private stages; frag: also the public
// stage of one half).
struct LpLdsPlan {
  size_t fixed, shared, per_wave;
};
LpLdsPlan lp_lds_plan(const Geom &g, int which) {
  const uint32_t npass = (g.npriv + 15u) / 16u, pstride = (2u * g.npriv * 64u + 15u) & ~15u;
  LpLdsPlan p;
  p.fixed = sizeof(AesLds) + (g.precision == SF_BF16 ? sizeof(LpLds<true>) : sizeof(LpLds<false>));
  p.shared = which == 0 ? 64u * npass * sizeof(LpQ2) : 0u;
  p.per_wave = (size_t)(which == 0 ? kFragGroup : kDefragGroup) * pstride + (which == 0 ? (size_t)64u * g.npub : 0u);
  return p;
}

// resident (the default): one resident generation of workgroups, each wave
// walking groups of tiles; otherwise one group of `group` tiles per wave.
int lp_grid(const DeviceState &ds, const void *kernel, const Shape &sh, size_t lds, uint32_t ntiles, uint32_t group) {
  const uint32_t w = sh.waves;
  if (!sh.resident) return (int)((ntiles + group * w - 1) / (group * w));
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 64 * (int)w, lds) != hipSuccess || per_cu < 1)
    per_cu = 1;
  const uint32_t need = (ntiles + w - 1) / w;
  const uint32_t cap = (uint32_t)ds.num_cu * (uint32_t)per_cu;
  return (int)(need < cap ? need : cap);
}

template <bool BF, class MP, bool kFrag>
int launch(const DeviceState &ds, const LpArgs &a0, const Shape &sh, const LpLdsPlan &p, hipStream_t stream) {
  LpArgs a = a0;
  const size_t lds = p.shared + (size_t)sh.waves * p.per_wave;
  a.wave_lds = (uint32_t)p.per_wave;
  const void *k = kFrag ? (const void *)&lp_frag_kernel<BF, MP> : (const void *)&lp_defrag_kernel<BF, MP>;
  const int grid = lp_grid(ds, k, sh, lds, a.g.ntiles, kFrag ? kFragGroup : kDefragGroup);
  if (kFrag)
    hipLaunchKernelGGL((lp_frag_kernel<BF, MP>), dim3(grid), dim3(64 * sh.waves), lds, stream, a);
  else
    hipLaunchKernelGGL((lp_defrag_kernel<BF, MP>), dim3(grid), dim3(64 * sh.waves), lds, stream, a);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SF_OK : hip_fail(e, kFrag ? "frag_lp kernel launch" : "defrag_lp kernel launch");
}

template <bool BF, bool kFrag>
int dispatch(const DeviceState &ds, const LpArgs &a, const Shape &sh, const LpLdsPlan &p, hipStream_t stream) {
  auto go = [&](auto mp) { return launch<BF, decltype(mp), kFrag>(ds, a, sh, p, stream); };
  switch (a.g.mask) {
    case (1ull << 2) - 1: return go(MaskPrefix<2>{});
    case (1ull << 3) - 1: return go(MaskPrefix<3>{});
    case (1ull << 6) - 1: return go(MaskPrefix<6>{});
    case (1ull << 10) - 1: return go(MaskPrefix<10>{});
    default: return go(MaskRuntime{});
  }
}

// The resolved shape, or SF_ENOTSUP if its LDS does not fit a workgroup.
int lp_shape(const DeviceState &ds, const Geom &g, int which, const Shape &in, Shape *out) {
  *out = in;
  if (!out->waves) {
    out->waves = lp_default_waves(ds, g, which);
    if (!out->waves) return fail(SF_ENOTSUP, "selection needs more LDS per workgroup than the device offers in this form");
  }
  if (out->waves > 8u || lp_lds_bytes(g, which, out->waves) > ds.max_lds_per_block)
    return fail(SF_ENOTSUP, "launch shape: the workgroup's LDS does not fit on this device");
  return SF_OK;
}

LpArgs lp_args(const DeviceState &ds, const Geom &g, const uint8_t *pix, const sf_exceptions *exc,
               const AesArgs &aes, uint32_t *status) {
  LpArgs a;
  memset(&a, 0, sizeof(a));
  a.g = tile_geom(g, pix);
  // every tile's count is written by frag: no clearing between calls
  const ExcLayout lay = exc_layout(g, exc->per_tile);
  uint8_t *eb = (uint8_t *)exc->d_buf;
  a.exc.count = (uint16_t *)eb;
  a.exc.pos = (uint16_t *)(eb + lay.pos_offset);
  a.exc.val = eb + lay.val_offset;
  a.exc.per_tile = exc->per_tile;
  a.exc.check = 1u;
  a.status = status;
  a.q2 = ds.d_q2;
  a.tables = ds.d_lp;
  a.aes_t0 = ds.d_aes_t0;
  a.aes = aes;
  a.npass = (g.npriv + 15u) / 16u;
  a.pstride = (2u * g.npriv * 64u + 15u) & ~15u;
  int i = 0;
  static constexpr ZigZag zz{};
  for (int z = 0; z < 64; ++z)
    if ((g.mask >> z) & 1u) {
      a.plist[i >> 2] |= (uint32_t)zz.nat[z] << (8 * (i & 3));
      ++i;
    }
  return a;
}

}  // namespace

size_t lp_lds_bytes(const Geom &g, int which, uint32_t waves) {
  const LpLdsPlan p = lp_lds_plan(g, which);
  return p.fixed + p.shared + (size_t)waves * p.per_wave;
}

// Waves per workgroup: the largest of 8, 6, 4, 2, 1 whose LDS leaves room for
// two workgroups per CU, else the largest that fits at all (0: none fits).
uint32_t lp_default_waves(const DeviceState &ds, const Geom &g, int which) {
  static const uint32_t cand[] = {8, 6, 4, 2, 1};
  const size_t cu_lds = 160u * 1024u;
  for (int pass = 0; pass < 2; ++pass)
    for (uint32_t w : cand) {
      const size_t b = lp_lds_bytes(g, which, w);
      if (b > ds.max_lds_per_block) continue;
      if (pass == 0 && 2 * b > cu_lds) continue;
      return w;
    }
  return 0;
}

int launch_frag_lp(const DeviceState &ds, const Geom &g, const uint8_t *pix, void *pub, uint8_t *priv,
                   const sf_exceptions *exc, uint8_t *residual, const AesArgs &aes, uint32_t *status,
                   const Shape &shape, hipStream_t stream) {
  Shape sh;
  if (int rc = lp_shape(ds, g, 0, shape, &sh)) return rc;
  LpArgs a = lp_args(ds, g, pix, exc, aes, status);
  a.pub = (uint16_t *)pub;
  a.priv = priv;
  a.resid = residual;
  const LpLdsPlan p = lp_lds_plan(g, 0);
  return g.precision == SF_BF16 ? dispatch<true, true>(ds, a, sh, p, stream)
                                : dispatch<false, true>(ds, a, sh, p, stream);
}

int launch_defrag_lp(const DeviceState &ds, const Geom &g, const void *pub, const uint8_t *priv,
                     const sf_exceptions *exc, const uint8_t *residual, const AesArgs &aes, uint8_t *pix,
                     uint32_t *status, const Shape &shape, hipStream_t stream) {
  Shape sh;
  if (int rc = lp_shape(ds, g, 1, shape, &sh)) return rc;
  LpArgs a = lp_args(ds, g, nullptr, exc, aes, status);
  a.pub = (uint16_t *)pub;
  a.priv = (uint8_t *)priv;
  a.resid = (uint8_t *)residual;
  a.pix_out = pix;
  const LpLdsPlan p = lp_lds_plan(g, 1);
  return g.precision == SF_BF16 ? dispatch<true, false>(ds, a, sh, p, stream)
                                : dispatch<false, false>(ds, a, sh, p, stream);
}

}  // namespace sf
