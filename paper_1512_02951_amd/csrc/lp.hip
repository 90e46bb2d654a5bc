// Reduced-precision form: the 8x8 DCT and inverse DCT as 64x64 basis
// contractions on the matrix cores (v_mfma_f32_32x32x16_{f16,bf16}, FP32
// accumulation), public coefficients stored as fp16 or bf16, private
// integers exactly as in the plain form, and a dense int8 residual plane
// r = x - clamp(round(IDCT(stored fragments))) that makes the round trip
// bit-exact.  frag computes the reconstruction with the same routine and the
// same operands defrag uses, so both see the same value bit for bit.
//
// One wavefront per tile of 64 blocks, processed as two 32-block halves
// (the N dimension of the MFMA).  Forward: C^T = K X^T with M = coefficient,
// N = block, K = pixel; inverse: X^T = K^T C^T with M = pixel.  bf16 keeps
// the basis as a hi + lo pair (and splits the private integers, which bf16
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
float f16_value(uint16_t b) {
  _Float16 h;
  memcpy(&h, &b, 2);
  return (float)h;
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

}  // namespace

// Table layout: word ((mt * 4 + s) * 64 + lane) * 4 + w holds elements
// e = 2w, 2w+1 of lane `lane` for M-tile mt and K-step s, i.e. the A operand
// of v_mfma_f32_32x32x16: row i = 32 mt + lane % 32, columns
// k = 16 s + 8 (lane / 32) + e.  Forward tables: A[i][k] = B[n = i][p = k];
// inverse tables: A[i][k] = B[n = k][p = i].
void build_lp_tables(const double *basis, uint32_t (*lp)[kLpTableWords]) {
  for (int inv = 0; inv < 2; ++inv)
    for (int mt = 0; mt < 2; ++mt)
      for (int s = 0; s < 4; ++s)
        for (int l = 0; l < 64; ++l)
          for (int e = 0; e < 8; ++e) {
            const int i = 32 * mt + (l & 31), k = 16 * s + 8 * (l >> 5) + e;
            const double v = inv ? basis[k * 64 + i] : basis[i * 64 + k];
            const uint16_t h16 = f16_bits(v);
            const uint16_t hb = bf16_bits(v);
            const uint16_t lb = bf16_bits(v - bf16_value(hb));
            (void)f16_value;
            const int word = ((mt * 4 + s) * 64 + l) * 4 + e / 2, sh = 16 * (e & 1);
            auto put = [&](int table, uint16_t bits) {
              if (sh == 0) lp[table][word] = 0u;
              lp[table][word] |= (uint32_t)bits << sh;
            };
            put(inv ? 1 : 0, h16);
            put(inv ? 4 : 2, hb);
            put(inv ? 5 : 3, lb);
          }
}

namespace {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;

// Waves per frag workgroup.  fp16 frag with a compile-time selection fits in
// 128 VGPRs (4 waves per SIMD), but the LDS of 4-wave workgroups admits only 3
// per CU; 8-wave workgroups fit 2 per CU, 16 waves.  The extra waves also even
// out the last round of tiles (an 8192^2 image: 4 tiles per wave instead of
// 5.33).  Every other kernel keeps 4-wave workgroups: measured, bf16 at 12
// waves per CU (6-wave workgroups) and fp16 defrag at 8 (8-wave workgroups,
// one per CU) ran 15-30 % slower than at their 8 and 12.
template <bool BF, class MP>
constexpr int frag_waves() {
  return (!BF && MP::kStatic) ? 8 : kWaves;
}

template <bool BF>
__device__ __forceinline__ f32x16 mfma(const uint4 &a, const uint4 &b, const f32x16 &c) {
  if constexpr (BF)
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0,
                                                   0, 0);
  else
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(half8, a), __builtin_bit_cast(half8, b), c, 0, 0,
                                                  0);
}

// 16-bit storage encodings (round to nearest even).
template <bool BF>
__device__ __forceinline__ uint32_t to16(float v) {
  if constexpr (BF) return (uint32_t)__builtin_bit_cast(uint16_t, (__bf16)v);
  else return (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)v);
}
template <bool BF>
__device__ __forceinline__ float from16(uint32_t b) {
  if constexpr (BF) return __uint_as_float(b << 16);
  else return (float)__builtin_bit_cast(_Float16, (uint16_t)b);
}

// Eight pixel bytes -> eight exact 16-bit values.
template <bool BF>
__device__ __forceinline__ uint4 pixels16(uint2 px) {
  uint32_t w[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const uint32_t src = i < 2 ? px.x : px.y;
    const float a = (float)((src >> (16 * (i & 1))) & 0xffu), b = (float)((src >> (16 * (i & 1) + 8)) & 0xffu);
    w[i] = to16<BF>(a) | (to16<BF>(b) << 16);
  }
  return make_uint4(w[0], w[1], w[2], w[3]);
}

// Operand tables in LDS (copied once per workgroup): per table
// 2 x 4 x 64 lanes x 16 bytes.
// f16: forward, inverse; bf16: forward hi, forward lo, inverse hi, inverse lo.
template <bool BF>
struct LpLds {
  static constexpr int kFwd = 0, kFwdLo = 1, kInv = BF ? 2 : 1, kInvLo = 3;
  uint4 t[BF ? 4 : 2][2 * 4 * 64];
};

template <bool BF>
__device__ __forceinline__ const uint4 &op(const LpLds<BF> &L, int table, int mt, int s, int lane) {
  return L.t[table][(mt * 4 + s) * 64 + lane];
}

// The one reconstruction routine: y[mt] (pixels 32 mt .. 32 mt + 31 of the
// lane's block column) = sum over K-steps of inverse basis x coefficients.
template <bool BF>
__device__ __forceinline__ void lp_idct(const LpLds<BF> &L, int lane, const uint4 (&chi)[4], const uint4 (&clo)[4],
                                        f32x16 (&y)[2]) {
#pragma unroll
  for (int mt = 0; mt < 2; ++mt) {
    f32x16 acc = {};
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      acc = mfma<BF>(op(L, LpLds<BF>::kInv, mt, s, lane), chi[s], acc);
      if constexpr (BF) {
        acc = mfma<BF>(op(L, LpLds<BF>::kInvLo, mt, s, lane), chi[s], acc);
        acc = mfma<BF>(op(L, LpLds<BF>::kInv, mt, s, lane), clo[s], acc);
      }
    }
    y[mt] = acc;
  }
}

// Rank bookkeeping for natural index n under a runtime mask (wave-uniform).
struct CoefSlot {
  uint32_t priv;  // 1 if private
  uint32_t rank;  // rank among the private (priv) or public (!priv) positions
};
__device__ __forceinline__ CoefSlot coef_slot(uint64_t mask, int n) {
  const int z = kZigZagInv.pos[n];
  const uint32_t before = (uint32_t)__builtin_popcountll(mask & ((1ull << z) - 1ull));
  CoefSlot c;
  c.priv = (uint32_t)((mask >> z) & 1u);
  c.rank = c.priv ? before : (uint32_t)z - before;
  return c;
}

// Private integer of natural index n -> (hi, lo) 16-bit operand pair.
template <bool BF>
__device__ __forceinline__ void split_int(int32_t q, uint32_t &hi, uint32_t &lo) {
  hi = to16<BF>((float)q);
  lo = BF ? to16<BF>((float)q - from16<BF>(hi)) : 0u;
}

struct LpFragArgs {
  TileGeom g;
  uint16_t *pub;
  uint8_t *priv;
  int8_t *resid;
  uint32_t *status;
  const uint32_t *q2;
  const uint32_t *tables;  // kLpTables x kLpTableWords
  const uint32_t *aes_t0;
  AesArgs aes;
  uint32_t lds_priv_bytes;
  uint32_t plist[16];      // natural indices of the private positions, 4 per word
};

struct LpDefragArgs {
  TileGeom g;
  const uint16_t *pub;
  const uint8_t *priv;
  const int8_t *resid;
  uint8_t *pix_out;
  uint32_t *status;
  const uint32_t *tables;
  const uint32_t *aes_t0;
  AesArgs aes;
  uint32_t lds_priv_bytes;
};

template <bool BF>
__device__ __forceinline__ void load_lp_tables(LpLds<BF> &L, const uint32_t *tables, int tid, int nthreads) {
  const uint4 *src = reinterpret_cast<const uint4 *>(tables);
  constexpr int kWords4 = kLpTableWords / 4;  // uint4 per table
  for (int i = tid; i < kWords4; i += nthreads) {
    if constexpr (BF) {
      L.t[0][i] = src[2 * kWords4 + i];
      L.t[1][i] = src[3 * kWords4 + i];
      L.t[2][i] = src[4 * kWords4 + i];
      L.t[3][i] = src[5 * kWords4 + i];
    } else {
      L.t[0][i] = src[0 * kWords4 + i];
      L.t[1][i] = src[1 * kWords4 + i];
    }
  }
}

// Coefficient bookkeeping of natural index n: compile-time for "DC + k AC"
// selections, wave-uniform otherwise.
template <class MP>
__device__ __forceinline__ CoefSlot slot_of(uint64_t mask, int n) {
  if constexpr (MP::kStatic) {
    const int z = kZigZagInv.pos[n];
    CoefSlot c;
    c.priv = z < MP::kNPriv ? 1u : 0u;
    c.rank = c.priv ? (uint32_t)z : (uint32_t)(z - MP::kNPriv);
    return c;
  } else {
    return coef_slot(mask, n);
  }
}

// Per-wave LDS: the tile's private integers (lds_priv_bytes), then a stage of
// kQ2StageBytes shared by the pixel staging of the quantiser, its
// accumulators, and the public values of one 32-block half (npub x 64 bytes).
constexpr uint32_t kLpStage = kQ2StageBytes;

// Public values of one half (stage rows of 64 bytes: rank r, block jl) to the
// tile-interleaved fragment, or back.  Full halves move 16 bytes per lane;
// a partial last tile moves element by element.
__device__ __forceinline__ void lp_public_out(uint16_t *pub_tile, const uint8_t *stage, uint32_t npub, uint32_t ntb,
                                              uint32_t nt, int lane) {
  const uint32_t nv = ntb > 32u * nt ? min(32u, ntb - 32u * nt) : 0u;
  if (nv == 32u && ntb == 64u) {
    for (uint32_t c = (uint32_t)lane; c < 4u * npub; c += 64u) {
      const uint32_t r = c >> 2, part = c & 3u;
      const uint4 v = *reinterpret_cast<const uint4 *>(stage + 64u * r + 16u * part);
      __builtin_nontemporal_store(v.x, reinterpret_cast<uint32_t *>(pub_tile + r * 64u + 32u * nt + 8u * part));
      __builtin_nontemporal_store(v.y, reinterpret_cast<uint32_t *>(pub_tile + r * 64u + 32u * nt + 8u * part + 2u));
      __builtin_nontemporal_store(v.z, reinterpret_cast<uint32_t *>(pub_tile + r * 64u + 32u * nt + 8u * part + 4u));
      __builtin_nontemporal_store(v.w, reinterpret_cast<uint32_t *>(pub_tile + r * 64u + 32u * nt + 8u * part + 6u));
    }
  } else {
    for (uint32_t c = (uint32_t)lane; c < 32u * npub; c += 64u) {
      const uint32_t r = c >> 5, j = c & 31u;
      if (j < nv) pub_tile[r * ntb + 32u * nt + j] = *reinterpret_cast<const uint16_t *>(stage + 64u * r + 2u * j);
    }
  }
}

// lp_public_in in two steps, so that the loads are in flight while other
// work runs: fetch (at most 4 x 16 bytes per lane for a full half; 63 ranks),
// then put into the stage rows.
struct LpPubFetch {
  uint4 v[4];
};

__device__ __forceinline__ LpPubFetch lp_public_fetch(const uint16_t *pub_tile, uint32_t npub, uint32_t ntb,
                                                      uint32_t nt, int lane) {
  LpPubFetch f;
  const uint32_t nv = ntb > 32u * nt ? min(32u, ntb - 32u * nt) : 0u;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    f.v[i] = make_uint4(0u, 0u, 0u, 0u);
    const uint32_t c = (uint32_t)lane + 64u * i;
    if (nv == 32u && ntb == 64u) {
      if (c < 4u * npub) {
        const uint32_t r = c >> 2, part = c & 3u;
        // default cache policy: the two halves of a tile read the two 64-byte
        // halves of each rank's 128-byte row, and a streaming hint would let
        // the second half fetch the line from HBM again
        f.v[i] = *reinterpret_cast<const uint4 *>(pub_tile + r * 64u + 32u * nt + 8u * part);
      }
    } else {
      // partial tile: chunk c covers rank c / 4, blocks 8 (c % 4) .. + 7 of this half
      if (c < 4u * npub) {
        const uint32_t r = c >> 2, j0 = 8u * (c & 3u);
        uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
        for (int j = 0; j < 8; ++j)
          if (j0 + j < nv) w[j >> 1] |= (uint32_t)pub_tile[r * ntb + 32u * nt + j0 + j] << (16 * (j & 1));
        f.v[i] = make_uint4(w[0], w[1], w[2], w[3]);
      }
    }
  }
  return f;
}

__device__ __forceinline__ void lp_public_put(const LpPubFetch &f, uint8_t *stage, uint32_t npub, int lane) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const uint32_t c = (uint32_t)lane + 64u * i;
    if (c < 4u * npub) *reinterpret_cast<uint4 *>(stage + 64u * (c >> 2) + 16u * (c & 3u)) = f.v[i];
  }
}

// Four reconstructed samples y[4 q4 .. 4 q4 + 3], rounded half to even and
// clamped to [0, 255] (v_cvt_pk_u8_f32), packed one per byte.
__device__ __forceinline__ uint32_t rec_word(const f32x16 &y, int q4) {
  uint32_t w = 0u;
#pragma unroll
  for (int e = 0; e < 4; ++e) w = __builtin_amdgcn_cvt_pk_u8_f32(y[4 * q4 + e], e, w);
  return w;
}

// Inverse-transform operands of one half: lane half h holds coefficients
// 16 s + 8 h + e (e = 0..7) of block jb; public ones are the stored 16-bit
// values (pub16(slot) returns them), private ones the integers from LDS,
// split into hi + lo for bf16.
template <bool BF, class MP, class PUB>
__device__ __forceinline__ void lp_inverse_operands(uint64_t mask, uint32_t h, uint32_t jb, bool bv, uint32_t ntb,
                                                    const uint8_t *lp, PUB &&pub16, uint4 (&chi)[4],
                                                    uint4 (&clo)[4]) {
  static_for<0, 4>([&](auto sc) {
    constexpr int s = decltype(sc)::value;
    uint32_t hi16[8], lo16[8];
    static_for<0, 8>([&](auto ec) {
      constexpr int e = decltype(ec)::value;
      constexpr int n0 = 16 * s + e, n1 = n0 + 8;
      const CoefSlot c0 = slot_of<MP>(mask, n0), c1 = slot_of<MP>(mask, n1);
      // both candidates are read without divergence (lane halves differ in
      // n); a read meant for the other half uses that half's own slot, so
      // every address stays in range
      const bool p0 = c0.priv != 0u, p1 = c1.priv != 0u;
      uint32_t hv = 0u, lv = 0u;
      if (p0 || p1) {
        const uint32_t rq = (p0 && p1) ? (h ? c1.rank : c0.rank) : (p0 ? c0.rank : c1.rank);
        const int32_t q = bv ? (int32_t) * reinterpret_cast<const int16_t *>(lp + 2u * (rq * ntb + jb)) : 0;
        split_int<BF>(q, hv, lv);
      }
      if (!p0 || !p1) {
        const uint32_t rp = (!p0 && !p1) ? (h ? c1.rank : c0.rank) : (!p0 ? c0.rank : c1.rank);
        const uint32_t pv = pub16(e, s, rp);
        if (p0 || p1) {
          const bool mine = h ? p1 : p0;  // this lane half's coefficient is private
          hv = mine ? hv : pv;
          lv = mine ? lv : 0u;
        } else {
          hv = pv;
        }
      }
      hi16[e] = hv;
      lo16[e] = lv;
    });
    chi[s] = make_uint4(hi16[0] | (hi16[1] << 16), hi16[2] | (hi16[3] << 16), hi16[4] | (hi16[5] << 16),
                        hi16[6] | (hi16[7] << 16));
    clo[s] = make_uint4(lo16[0] | (lo16[1] << 16), lo16[2] | (lo16[3] << 16), lo16[4] | (lo16[5] << 16),
                        lo16[6] | (lo16[7] << 16));
  });
}

// Pixel words of one half in the residual layout: the forward operand rows
// (lane half h: rows 2s + h, 8 bytes) rearranged so that lane half h holds
// columns 4h..4h+3 of every row r in row[r].
__device__ __forceinline__ void lp_pixel_rows(const uint2 (&prow)[4], uint32_t (&row)[8]) {
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    // lanes 0-31 hold row 2s, lanes 32-63 row 2s+1 (x: columns 0-3, y:
    // columns 4-7).  Swapping x of lanes 32-63 with y of lanes 0-31 leaves
    // row 2s in x and row 2s+1 in y, columns 0-3 in lanes 0-31 and 4-7 in
    // lanes 32-63.
    const auto sw = __builtin_amdgcn_permlane32_swap(prow[s].x, prow[s].y, false, false);
    row[2 * s] = sw[0];
    row[2 * s + 1] = sw[1];
  }
}

template <bool BF, class MP, bool kQ2Mfma>
__global__ __launch_bounds__(64 * (frag_waves<BF, MP>()), MP::kStatic ? 3 : 2) void frag_lp_kernel(LpFragArgs a) {
  constexpr uint32_t nw = frag_waves<BF, MP>();
  __shared__ AesLds s_aes;
  __shared__ LpLds<BF> s_tab;
  __shared__ Q2Operands s_q2[kQ2Mfma ? 64 : 1];
  extern __shared__ __attribute__((aligned(16))) uint8_t s_dyn[];
  const int lane = threadIdx.x & 63;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const TileGeom &g = a.g;
  if (a.aes.enabled) aes_load_tables(s_aes, a.aes_t0, a.aes.key, threadIdx.x, 64 * nw);
  load_lp_tables<BF>(s_tab, a.tables, threadIdx.x, 64 * nw);
  if constexpr (kQ2Mfma)
    if (threadIdx.x < 64) s_q2[lane] = q2_operands(a.q2, private_ac<MP>(g.mask, lane & 15), lane);
  __syncthreads();
  uint8_t *lp = s_dyn + wave * (a.lds_priv_bytes + kLpStage);
  uint8_t *stage = lp + a.lds_priv_bytes;
  const uint64_t mask = MP::kStatic ? g.mask : opaque_u64(g.mask);
  const uint32_t h = (uint32_t)lane >> 5, jl = (uint32_t)lane & 31u;
  const uint32_t stride = gridDim.x * nw;
  uint32_t rflag = 0;

  uint32_t t = blockIdx.x * nw + wave;
  TileLane Lnext = tile_lane(g, t < g.ntiles ? t : 0u, lane);
  uint32_t xs[16];
  if (t < g.ntiles) load_block(g, Lnext, xs);
  for (; t < g.ntiles; t += stride) {
    const TileLane L = Lnext;
    const uint64_t b0 = L.b0;
    const uint32_t ntb = L.nt;
    const uint32_t tn = t + stride;

    // ---- the lane's block: exact sum, staged for the quantiser and for the
    // forward-transform operands (lane half h: rows 2s + h of block jb)
    uint2 prow[2][4];
    {
      uint32_t S = 0;
#pragma unroll
      for (int w = 0; w < 16; ++w) S = __builtin_amdgcn_udot4(xs[w], 0x01010101u, S, false);
#pragma unroll
      for (int w = 0; w < 16; ++w) xs[w] ^= 0x80808080u;
      q2_stage_pixels(xs, lane, stage);
      wave_lds_sync();
#pragma unroll
      for (int nt = 0; nt < 2; ++nt)
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const uint2 v = *reinterpret_cast<const uint2 *>(stage + (32u * nt + jl) * kQ2PixStride + (2u * s + h) * 8u);
          prow[nt][s] = make_uint2(v.x ^ 0x80808080u, v.y ^ 0x80808080u);
        }
      const cu32_ptr q2 = as_const(a.q2) + opaque_zero();
      if constexpr (kQ2Mfma) {
        q2v4 A[4];
        q2_read_a(lane, stage, A);
        wave_lds_sync();
        q2_products(A, lane, stage, s_q2[lane]);
        wave_lds_sync();
      }
      // ---- private integers, one block per lane (as in the plain form)
      const uint32_t dc_priv = (uint32_t)(mask & 1u);
      for (uint32_t i = 0; i < g.npriv; ++i) {
        const uint32_t n = (a.plist[i >> 2] >> (8 * (i & 3))) & 0xffu;
        int32_t q;
        if (n == 0) q = (int32_t)((S + 3u + ((S >> 3) & 1u)) >> 3);
        else if constexpr (kQ2Mfma) q = q2_round(q2_mfma_acc(stage, i - dc_priv, lane));
        else q = q2_round(q2_acc(xs, q2 + n * kQ2RowWords));
        if (L.valid) *reinterpret_cast<int16_t *>(lp + 2u * (i * ntb + lane)) = (int16_t)q;
      }
      // the next tile's pixels, in flight during the transforms of this one
      if (tn < g.ntiles) {
        Lnext = tile_lane(g, tn, lane);
        load_block(g, Lnext, xs);
      }
    }
    wave_lds_sync();

    uint16_t *pub_tile = a.pub + b0 * g.npub;
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
      const uint32_t jb = 32u * nt + jl;
      const bool bv = jb < ntb;
      const uint32_t borg = bv ? block_origin(g, (uint32_t)b0 + jb) : 0u;

      // ---- forward transform: C^T = K X^T
      f32x16 acc[2];
      {
        uint4 bx[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) bx[s] = pixels16<BF>(prow[nt][s]);
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

      // ---- stored 16-bit values; public ones to the stage rows
      uint32_t bits[2][16];
      static_for<0, 2>([&](auto mtc) {
        constexpr int mt = decltype(mtc)::value;
        static_for<0, 16>([&](auto rc) {
          constexpr int r = decltype(rc)::value;
          constexpr int n0 = 32 * mt + 8 * (r >> 2) + (r & 3), n1 = n0 + 4;
          const CoefSlot c0 = slot_of<MP>(mask, n0), c1 = slot_of<MP>(mask, n1);
          const uint32_t priv = h ? c1.priv : c0.priv, rank = h ? c1.rank : c0.rank;
          const uint32_t b = to16<BF>(acc[mt][r]);
          bits[mt][r] = b;
          if (!priv) *reinterpret_cast<uint16_t *>(stage + 64u * rank + 2u * jl) = (uint16_t)(bv ? b : 0u);
        });
      });

      // ---- inverse-transform operands: exchange lane halves so lane half h
      // holds coefficients 16 s + 8 h + e (e = 0..7) of its block
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int sl = 0; sl < 2; ++sl)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const auto sw = __builtin_amdgcn_permlane32_swap(bits[mt][8 * sl + e], bits[mt][8 * sl + 4 + e], false, false);
            bits[mt][8 * sl + e] = sw[0];
            bits[mt][8 * sl + 4 + e] = sw[1];
          }
      uint4 chi[4], clo[4];
      lp_inverse_operands<BF, MP>(mask, h, jb, bv, ntb, lp,
                                  [&](int e, int s, uint32_t) { return bits[s / 2][8 * (s & 1) + e]; }, chi, clo);

      // ---- reconstruction and residual plane
      uint32_t row[8];
      lp_pixel_rows(prow[nt], row);
      f32x16 y[2];
      lp_idct<BF>(s_tab, lane, chi, clo, y);
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int q4 = 0; q4 < 4; ++q4) {
          const uint32_t xw = row[4 * mt + q4];
          const uint32_t rec = rec_word(y[mt], q4);
          const uint32_t rw = bytes_sub(xw, rec);
          // every |x - rec| <= 127 when their sum is; otherwise check each byte
          if (__builtin_amdgcn_sad_u8(xw, rec, 0u) > 127u) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const int d = (int)((xw >> (8 * e)) & 0xffu) - (int)((rec >> (8 * e)) & 0xffu);
              rflag |= (d < -128 || d > 127) ? 1u : 0u;
            }
          }
          if (bv)
            __builtin_nontemporal_store(rw, reinterpret_cast<uint32_t *>(a.resid + borg + (size_t)(4 * mt + q4) * g.W + 4u * h));
        }

      // ---- this half's public values, 16 bytes per lane
      wave_lds_sync();
      lp_public_out(pub_tile, stage, g.npub, ntb, (uint32_t)nt, lane);
      wave_lds_sync();
    }

    // ---- private bytes: AES-CTR and coalesced stores
    tile_ctr_store(lp, a.priv + b0 * g.npriv * 2u, 2u * g.npriv * ntb, lane, s_aes, a.aes.enabled, a.aes.ctr_hi,
                   a.aes.ctr_lo, b0 * g.npriv / 8u);
    wave_lds_sync();
  }
  if (__ballot(rflag != 0u) != 0ull && lane == 0 && a.status) atomicOr(a.status, SF_STATUS_RESIDUAL_RANGE);
}

template <bool BF, class MP>
__global__ __launch_bounds__(kThreads, MP::kStatic ? 3 : 2) void defrag_lp_kernel(LpDefragArgs a) {
  __shared__ AesLds s_aes;
  __shared__ LpLds<BF> s_tab;
  extern __shared__ __attribute__((aligned(16))) uint8_t s_dyn[];
  const int lane = threadIdx.x & 63;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (a.aes.enabled) aes_load_tables(s_aes, a.aes_t0, a.aes.key, threadIdx.x, kThreads);
  load_lp_tables<BF>(s_tab, a.tables, threadIdx.x, kThreads);
  __syncthreads();
  uint8_t *lp = s_dyn + wave * (a.lds_priv_bytes + kLpStage);
  uint8_t *stage = lp + a.lds_priv_bytes;
  const TileGeom &g = a.g;
  const uint64_t mask = MP::kStatic ? g.mask : opaque_u64(g.mask);
  const uint32_t h = (uint32_t)lane >> 5, jl = (uint32_t)lane & 31u;
  const uint32_t stride = gridDim.x * kWaves;

  for (uint32_t t = blockIdx.x * kWaves + wave; t < g.ntiles; t += stride) {
    const uint64_t b0 = (uint64_t)t * 64u;
    const uint32_t ntb = (uint32_t)min<uint64_t>(64u, g.nb - b0);
    const uint16_t *pub_tile = a.pub + b0 * g.npub;
    LpPubFetch pf = lp_public_fetch(pub_tile, g.npub, ntb, 0u, lane);  // in flight during the AES pass
    tile_ctr_load(lp, a.priv + b0 * g.npriv * 2u, 2u * g.npriv * ntb, lane, s_aes, a.aes.enabled, a.aes.ctr_hi,
                  a.aes.ctr_lo, b0 * g.npriv / 8u);
    lp_public_put(pf, stage, g.npub, lane);
    wave_lds_sync();
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
      const uint32_t jb = 32u * nt + jl;
      const bool bv = jb < ntb;
      const uint32_t borg = bv ? block_origin(g, (uint32_t)b0 + jb) : 0u;
      // this half's residual words, in flight during the operand gathering and
      // the inverse transform
      uint32_t rw[8];
#pragma unroll
      for (int r = 0; r < 8; ++r)
        rw[r] = bv ? __builtin_nontemporal_load(reinterpret_cast<const uint32_t *>(a.resid + borg + (size_t)r * g.W + 4u * h))
                   : 0u;
      uint4 chi[4], clo[4];
      lp_inverse_operands<BF, MP>(mask, h, jb, bv, ntb, lp,
                                  [&](int, int, uint32_t rank) {
                                    return (uint32_t) * reinterpret_cast<const uint16_t *>(stage + 64u * rank + 2u * jl);
                                  },
                                  chi, clo);
      if (nt == 0) pf = lp_public_fetch(pub_tile, g.npub, ntb, 1u, lane);  // next half, in flight during the IDCT
      f32x16 y[2];
      lp_idct<BF>(s_tab, lane, chi, clo, y);
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int q4 = 0; q4 < 4; ++q4) {
          const size_t off = borg + (size_t)(4 * mt + q4) * g.W + 4u * h;
          // rec + r is the sample itself, in [0, 255]: byte-wise addition
          const uint32_t ow = bytes_add(rec_word(y[mt], q4), rw[4 * mt + q4]);
          if (bv) __builtin_nontemporal_store(ow, reinterpret_cast<uint32_t *>(a.pix_out + off));
        }
      if (nt == 0) {
        wave_lds_sync();
        lp_public_put(pf, stage, g.npub, lane);
        wave_lds_sync();
      }
    }
    wave_lds_sync();
  }
}

uint32_t lds_priv_bytes(const Geom &g) { return (2u * g.npriv * 64u + 15u) & ~15u; }

int grid_for(const DeviceState &ds, const void *kernel, int waves, size_t lds, uint32_t ntiles) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 64 * waves, lds) != hipSuccess || per_cu < 1)
    per_cu = 1;
  const uint32_t need = (ntiles + waves - 1) / waves;
  const uint32_t cap = (uint32_t)ds.num_cu * (uint32_t)per_cu;
  return (int)(need < cap ? need : cap);
}

template <bool BF>
int lds_fits(const DeviceState &ds, size_t dynamic) {
  const size_t total = sizeof(AesLds) + sizeof(LpLds<BF>) + 64 * sizeof(Q2Operands) + dynamic;
  if (total > ds.max_lds_per_block)
    return fail(SF_ENOTSUP, "selection needs more LDS per workgroup than the device offers in this form");
  return SF_OK;
}

template <bool BF, class MP, bool kQ2Mfma>
int launch_frag(const DeviceState &ds, const LpFragArgs &a, hipStream_t stream) {
  constexpr int nw = frag_waves<BF, MP>();
  const size_t lds = (size_t)nw * (a.lds_priv_bytes + kLpStage);
  if (int rc = lds_fits<BF>(ds, lds)) return rc;
  const int grid = grid_for(ds, (const void *)&frag_lp_kernel<BF, MP, kQ2Mfma>, nw, lds, a.g.ntiles);
  hipLaunchKernelGGL((frag_lp_kernel<BF, MP, kQ2Mfma>), dim3(grid), dim3(64 * nw), lds, stream, a);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SF_OK : hip_fail(e, "frag_lp kernel launch");
}

template <bool BF, class MP>
int launch_defrag(const DeviceState &ds, const LpDefragArgs &a, hipStream_t stream) {
  const size_t lds = (size_t)kWaves * (a.lds_priv_bytes + kLpStage);
  if (int rc = lds_fits<BF>(ds, lds)) return rc;
  const int grid = grid_for(ds, (const void *)&defrag_lp_kernel<BF, MP>, kWaves, lds, a.g.ntiles);
  hipLaunchKernelGGL((defrag_lp_kernel<BF, MP>), dim3(grid), dim3(kThreads), lds, stream, a);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SF_OK : hip_fail(e, "defrag_lp kernel launch");
}

template <bool BF>
int dispatch_frag(const DeviceState &ds, const LpFragArgs &a, hipStream_t stream) {
  switch (a.g.mask) {
    case (1ull << 2) - 1: return launch_frag<BF, MaskPrefix<2>, true>(ds, a, stream);
    case (1ull << 3) - 1: return launch_frag<BF, MaskPrefix<3>, true>(ds, a, stream);
    case (1ull << 6) - 1: return launch_frag<BF, MaskPrefix<6>, true>(ds, a, stream);
    case (1ull << 10) - 1: return launch_frag<BF, MaskPrefix<10>, true>(ds, a, stream);
    default:
      if (__builtin_popcountll(a.g.mask & ~1ull) <= kQ2MfmaMaxAc) return launch_frag<BF, MaskRuntime, true>(ds, a, stream);
      return launch_frag<BF, MaskRuntime, false>(ds, a, stream);
  }
}

template <bool BF>
int dispatch_defrag(const DeviceState &ds, const LpDefragArgs &a, hipStream_t stream) {
  switch (a.g.mask) {
    case (1ull << 2) - 1: return launch_defrag<BF, MaskPrefix<2>>(ds, a, stream);
    case (1ull << 3) - 1: return launch_defrag<BF, MaskPrefix<3>>(ds, a, stream);
    case (1ull << 6) - 1: return launch_defrag<BF, MaskPrefix<6>>(ds, a, stream);
    case (1ull << 10) - 1: return launch_defrag<BF, MaskPrefix<10>>(ds, a, stream);
    default: return launch_defrag<BF, MaskRuntime>(ds, a, stream);
  }
}

}  // namespace

int launch_frag_lp(const DeviceState &ds, const Geom &g, const uint8_t *pix, void *pub, uint8_t *priv,
                   int8_t *residual, const AesArgs &aes, uint32_t *status, hipStream_t stream) {
  LpFragArgs a;
  a.g = tile_geom(g, pix);
  a.pub = (uint16_t *)pub;
  a.priv = priv;
  a.resid = residual;
  a.status = status;
  a.q2 = ds.d_q2;
  a.tables = ds.d_lp;
  a.aes_t0 = ds.d_aes_t0;
  a.aes = aes;
  a.lds_priv_bytes = lds_priv_bytes(g);
  memset(a.plist, 0, sizeof(a.plist));
  int i = 0;
  static constexpr ZigZag zz{};
  for (int z = 0; z < 64; ++z)
    if ((g.mask >> z) & 1u) {
      a.plist[i >> 2] |= (uint32_t)zz.nat[z] << (8 * (i & 3));
      ++i;
    }
  return g.precision == SF_BF16 ? dispatch_frag<true>(ds, a, stream) : dispatch_frag<false>(ds, a, stream);
}

int launch_defrag_lp(const DeviceState &ds, const Geom &g, const void *pub, const uint8_t *priv,
                     const int8_t *residual, const AesArgs &aes, uint8_t *pix, uint32_t *status,
                     hipStream_t stream) {
  LpDefragArgs a;
  a.g = tile_geom(g, nullptr);
  a.pub = (const uint16_t *)pub;
  a.priv = priv;
  a.resid = residual;
  a.pix_out = pix;
  a.status = status;
  a.tables = ds.d_lp;
  a.aes_t0 = ds.d_aes_t0;
  a.aes = aes;
  a.lds_priv_bytes = lds_priv_bytes(g);
  return g.precision == SF_BF16 ? dispatch_defrag<true>(ds, a, stream) : dispatch_defrag<false>(ds, a, stream);
}

}  // namespace sf
