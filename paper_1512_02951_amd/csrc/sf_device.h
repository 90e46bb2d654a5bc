// Device building blocks shared by every kernel of the library: the 8x8
// DCT-II / inverse DCT butterflies in FP32, the JPEG zigzag table, the
// integer private quantiser and AES-128 round functions on LDS tables.
//
// Floating-point contraction is disabled for this whole translation unit
// family: every fused multiply-add below is written explicitly, so that the
// reconstruction computed during fragmentation (to find exceptions) and the
// one computed during defragmentation are the same IEEE operations on the
// same operands and therefore bit-identical.
#pragma once
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>

namespace sf {

// ---------------------------------------------------------------------------
// Compile-time loops (indices stay constants, so register arrays are never
// indexed dynamically).
template <int Begin, int End, typename F>
__device__ __forceinline__ void static_for(F &&f) {
  if constexpr (Begin < End) {
    f(std::integral_constant<int, Begin>{});
    static_for<Begin + 1, End>(static_cast<F &&>(f));
  }
}

// ---------------------------------------------------------------------------
// JPEG zigzag: zigzag position z -> natural index 8u + v.  Built by walking
// the anti-diagonals; on odd diagonals the row index grows.
struct ZigZag {
  int nat[64];
  constexpr ZigZag() : nat{} {
    int z = 0;
    for (int d = 0; d < 15; ++d) {
      int lo = d < 8 ? 0 : d - 7, hi = d < 8 ? d : 7;
      for (int i = 0; i <= hi - lo; ++i) {
        int u = (d & 1) ? lo + i : hi - i;
        nat[z++] = 8 * u + (d - u);
      }
    }
  }
};
inline constexpr ZigZag kZigZag{};

// Inverse table: natural index 8u + v -> zigzag position.
struct ZigZagInv {
  int pos[64];
  constexpr ZigZagInv() : pos{} {
    for (int z = 0; z < 64; ++z) pos[kZigZag.nat[z]] = z;
  }
};
inline constexpr ZigZagInv kZigZagInv{};

// ---------------------------------------------------------------------------
// Orthonormal 8-point DCT-II constants (host computes them; see tables.cpp):
//   s0 = 1/sqrt(8), a = cos(pi/8)/2, b = cos(3pi/8)/2, cK = cos(K pi/16)/2.
struct DctK {
  float s0, a, b, c1, c3, c5, c7;
};

// Forward 8-point DCT (even/odd butterfly):
//   X_u = sum_i d[u][i] x_i with d[u][i] = c(u) cos((2i+1) u pi / 16).
__device__ __forceinline__ void fdct8(float &x0, float &x1, float &x2, float &x3, float &x4, float &x5,
                                      float &x6, float &x7, const DctK &K) {
  const float s0 = x0 + x7, s1 = x1 + x6, s2 = x2 + x5, s3 = x3 + x4;
  const float t0 = x0 - x7, t1 = x1 - x6, t2 = x2 - x5, t3 = x3 - x4;
  const float p0 = s0 + s3, p1 = s1 + s2, m0 = s0 - s3, m1 = s1 - s2;
  x0 = K.s0 * (p0 + p1);
  x4 = K.s0 * (p0 - p1);
  x2 = __builtin_fmaf(K.a, m0, K.b * m1);
  x6 = __builtin_fmaf(K.b, m0, -(K.a * m1));
  x1 = __builtin_fmaf(K.c1, t0, __builtin_fmaf(K.c3, t1, __builtin_fmaf(K.c5, t2, K.c7 * t3)));
  x3 = __builtin_fmaf(K.c3, t0, __builtin_fmaf(-K.c7, t1, __builtin_fmaf(-K.c1, t2, -(K.c5 * t3))));
  x5 = __builtin_fmaf(K.c5, t0, __builtin_fmaf(-K.c1, t1, __builtin_fmaf(K.c7, t2, K.c3 * t3)));
  x7 = __builtin_fmaf(K.c7, t0, __builtin_fmaf(-K.c5, t1, __builtin_fmaf(K.c3, t2, -(K.c1 * t3))));
}

// Inverse 8-point DCT: x_i = sum_u d[u][i] X_u.
__device__ __forceinline__ void idct8(float &x0, float &x1, float &x2, float &x3, float &x4, float &x5,
                                      float &x6, float &x7, const DctK &K) {
  const float E0 = K.s0 * (x0 + x4), E1 = K.s0 * (x0 - x4);
  const float F0 = __builtin_fmaf(K.a, x2, K.b * x6), F1 = __builtin_fmaf(K.b, x2, -(K.a * x6));
  const float e0 = E0 + F0, e3 = E0 - F0, e1 = E1 + F1, e2 = E1 - F1;
  const float o0 = __builtin_fmaf(K.c1, x1, __builtin_fmaf(K.c3, x3, __builtin_fmaf(K.c5, x5, K.c7 * x7)));
  const float o1 = __builtin_fmaf(K.c3, x1, __builtin_fmaf(-K.c7, x3, __builtin_fmaf(-K.c1, x5, -(K.c5 * x7))));
  const float o2 = __builtin_fmaf(K.c5, x1, __builtin_fmaf(-K.c1, x3, __builtin_fmaf(K.c7, x5, K.c3 * x7)));
  const float o3 = __builtin_fmaf(K.c7, x1, __builtin_fmaf(-K.c5, x3, __builtin_fmaf(K.c3, x5, -(K.c1 * x7))));
  x0 = e0 + o0;
  x7 = e0 - o0;
  x1 = e1 + o1;
  x6 = e1 - o1;
  x2 = e2 + o2;
  x5 = e2 - o2;
  x3 = e3 + o3;
  x4 = e3 - o3;
}

// 2-D forward DCT of one block held as c[8y + x] -> c[8u + v]:
// rows (over x) then columns (over y).
__device__ __forceinline__ void fdct8x8(float (&c)[64], const DctK &K) {
  static_for<0, 8>([&](auto y) {
    constexpr int r = 8 * decltype(y)::value;
    fdct8(c[r + 0], c[r + 1], c[r + 2], c[r + 3], c[r + 4], c[r + 5], c[r + 6], c[r + 7], K);
  });
  static_for<0, 8>([&](auto v) {
    constexpr int q = decltype(v)::value;
    fdct8(c[q], c[q + 8], c[q + 16], c[q + 24], c[q + 32], c[q + 40], c[q + 48], c[q + 56], K);
  });
}

// 2-D inverse DCT c[8u + v] -> c[8y + x]: columns (over u) then rows (over v).
// This is the one reconstruction routine of the library.
__device__ __forceinline__ void idct8x8(float (&c)[64], const DctK &K) {
  static_for<0, 8>([&](auto v) {
    constexpr int q = decltype(v)::value;
    idct8(c[q], c[q + 8], c[q + 16], c[q + 24], c[q + 32], c[q + 40], c[q + 48], c[q + 56], K);
  });
  static_for<0, 8>([&](auto y) {
    constexpr int r = 8 * decltype(y)::value;
    idct8(c[r + 0], c[r + 1], c[r + 2], c[r + 3], c[r + 4], c[r + 5], c[r + 6], c[r + 7], K);
  });
}

// ---------------------------------------------------------------------------
// Integer private quantiser.  With Bq[n][p] = rhe(2^20 B[n][p]) split into
// signed bytes Bq = h*2^16 + m*2^8 + l, and x_p = (x_p - 128) + 128:
//   acc = 2^16 D_h + 2^8 D_m + D_l + 128 * sum_p Bq[n][p],
// D_* = sum_p (x_p - 128) * limb_p, evaluated with 4-way int8 dot products on
// the packed pixel words.  All arithmetic is modulo 2^32; the exact result
// |acc| <= 2040 * 2^20 < 2^31 fits, so the wrapped value is exact.
// Table row layout (kQ2RowWords words per natural index n):
//   [0,16) limb l, [16,32) limb m, [32,48) limb h (4 signed bytes per word,
//   byte i of word w is pixel p = 4w + i), [48] = 128 * sum_p Bq[n][p],
//   [49] = E_n as float bits: 255 * sum_p |Bq[n][p]/2^20 - B[n][p]| (>= |acc/2^20 - C_n|),
//   [50] = M_n as float bits: max_p |B[n][p]| (both rounded up).
constexpr int kQ2RowWords = 52;
constexpr int kQ2CertE = 49;
constexpr int kQ2CertM = 50;

// Read-only tables are read through constant-address-space pointers so that
// wave-uniform reads become scalar loads into SGPRs.
typedef const uint32_t __attribute__((address_space(4))) *cu32_ptr;
__device__ __forceinline__ cu32_ptr as_const(const uint32_t *p) { return (cu32_ptr)(uintptr_t)p; }

// A zero the compiler cannot see through: adding it to a table address inside
// a loop keeps the (scalar) table loads in the loop instead of hoisting
// thousands of loop-invariant values into registers.
__device__ __forceinline__ uint32_t opaque_zero() {
  uint32_t z = 0;
  asm volatile("" : "+s"(z));
  return z;
}

__device__ __forceinline__ int32_t q2_acc(const uint32_t (&xs)[16], cu32_ptr row) {
  int dl = 0, dm = 0, dh = 0;
#pragma unroll
  for (int w = 0; w < 16; ++w) {
    dl = __builtin_amdgcn_sdot4((int)xs[w], (int)row[w], dl, false);
    dm = __builtin_amdgcn_sdot4((int)xs[w], (int)row[16 + w], dm, false);
    dh = __builtin_amdgcn_sdot4((int)xs[w], (int)row[32 + w], dh, false);
  }
  uint32_t acc = ((uint32_t)dh << 16) + ((uint32_t)dm << 8) + (uint32_t)dl + row[48];
  return (int32_t)acc;
}

// round half to even of acc / 2^20 (arithmetic shifts are floors).
__device__ __forceinline__ int32_t q2_round(int32_t acc) {
  return (acc + (1 << 19) - 1 + ((acc >> 20) & 1)) >> 20;
}

// ---------------------------------------------------------------------------
// AES-128 (FIPS-197) with the classic 32-bit table formulation: one round of
// SubBytes+ShiftRows+MixColumns on state column j is
//   T0[s_j.b0] ^ T1[s_{j+1}.b1] ^ T2[s_{j+2}.b2] ^ T3[s_{j+3}.b3] ^ rk,
// columns as little-endian words (byte r = state row r).  T1..T3 are byte
// rotations of T0; the final round takes the S-box byte out of the tables.
struct AesKey {
  uint32_t rk[44];  // expanded key, little-endian words
};

// Round tables and the expanded key, copied into LDS once per workgroup
// (the key is read with wave-uniform broadcasts).
struct AesLds {
  uint32_t t[4][256];
  uint32_t rk[44];
};

__device__ __forceinline__ void aes_load_tables(AesLds &L, const uint32_t *__restrict__ T0, const AesKey &K, int tid,
                                                int nthreads) {
  for (int i = tid; i < 256; i += nthreads) {
    uint32_t v = T0[i];
    L.t[0][i] = v;
    L.t[1][i] = (v << 8) | (v >> 24);
    L.t[2][i] = (v << 16) | (v >> 16);
    L.t[3][i] = (v << 24) | (v >> 8);
  }
  for (int i = tid; i < 44; i += nthreads) L.rk[i] = K.rk[i];
}

// The lane index from an opaque instruction pair: values derived from it are
// computed where they are used rather than held (or spilled) across a whole
// kernel from its entry.
__device__ __forceinline__ uint32_t fresh_lane() {
  uint32_t l;
  asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0" : "=v"(l));
  return l;
}

__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);  // truth table of a ^ b ^ c
}

// Byte-wise a - b and a + b modulo 256 (no carry or borrow between bytes).
__device__ __forceinline__ uint32_t bytes_sub(uint32_t a, uint32_t b) {
  return ((a | 0x80808080u) - (b & 0x7f7f7f7fu)) ^ ((a ^ ~b) & 0x80808080u);
}
__device__ __forceinline__ uint32_t bytes_add(uint32_t a, uint32_t b) {
  return ((a & 0x7f7f7f7fu) + (b & 0x7f7f7f7fu)) ^ ((a ^ b) & 0x80808080u);
}

// One AES-128 encryption (FIPS-197 Sec. 5.1) of the state words s0..s3 with
// the T-table formulation: each middle round is 16 table lookups whose byte
// indices the compiler takes with sub-dword operand selection, and two
// three-input XORs per column.
__device__ __forceinline__ void aes_encrypt(uint32_t &s0, uint32_t &s1, uint32_t &s2, uint32_t &s3,
                                            const AesLds &L) {
  const uint32_t *rk = L.rk;
  s0 ^= rk[0];
  s1 ^= rk[1];
  s2 ^= rk[2];
  s3 ^= rk[3];
#pragma unroll
  for (int r = 1; r < 10; ++r) {
    const uint32_t t0 = xor3(xor3(L.t[0][s0 & 0xff], L.t[1][(s1 >> 8) & 0xff], L.t[2][(s2 >> 16) & 0xff]),
                             L.t[3][s3 >> 24], rk[4 * r]);
    const uint32_t t1 = xor3(xor3(L.t[0][s1 & 0xff], L.t[1][(s2 >> 8) & 0xff], L.t[2][(s3 >> 16) & 0xff]),
                             L.t[3][s0 >> 24], rk[4 * r + 1]);
    const uint32_t t2 = xor3(xor3(L.t[0][s2 & 0xff], L.t[1][(s3 >> 8) & 0xff], L.t[2][(s0 >> 16) & 0xff]),
                             L.t[3][s1 >> 24], rk[4 * r + 2]);
    const uint32_t t3 = xor3(xor3(L.t[0][s3 & 0xff], L.t[1][(s0 >> 8) & 0xff], L.t[2][(s1 >> 16) & 0xff]),
                             L.t[3][s2 >> 24], rk[4 * r + 3]);
    s0 = t0;
    s1 = t1;
    s2 = t2;
    s3 = t3;
  }
  // last round: S-box byte r sits at byte r of T2, T3, T0, T1 for r = 0..3
  const uint32_t t0 = (L.t[2][s0 & 0xff] & 0x000000ffu) | (L.t[3][(s1 >> 8) & 0xff] & 0x0000ff00u) |
                      (L.t[0][(s2 >> 16) & 0xff] & 0x00ff0000u) | (L.t[1][s3 >> 24] & 0xff000000u);
  const uint32_t t1 = (L.t[2][s1 & 0xff] & 0x000000ffu) | (L.t[3][(s2 >> 8) & 0xff] & 0x0000ff00u) |
                      (L.t[0][(s3 >> 16) & 0xff] & 0x00ff0000u) | (L.t[1][s0 >> 24] & 0xff000000u);
  const uint32_t t2 = (L.t[2][s2 & 0xff] & 0x000000ffu) | (L.t[3][(s3 >> 8) & 0xff] & 0x0000ff00u) |
                      (L.t[0][(s0 >> 16) & 0xff] & 0x00ff0000u) | (L.t[1][s1 >> 24] & 0xff000000u);
  const uint32_t t3 = (L.t[2][s3 & 0xff] & 0x000000ffu) | (L.t[3][(s0 >> 8) & 0xff] & 0x0000ff00u) |
                      (L.t[0][(s1 >> 16) & 0xff] & 0x00ff0000u) | (L.t[1][s2 >> 24] & 0xff000000u);
  s0 = t0 ^ rk[40];
  s1 = t1 ^ rk[41];
  s2 = t2 ^ rk[42];
  s3 = t3 ^ rk[43];
}

// Column c of state word s from lane (lane & ~3) + ((lane + K) & 3) of the
// same quad (DPP quad permute; every lane of the quad must be active).
template <int K>
__device__ __forceinline__ uint32_t quad_next(uint32_t s) {
  constexpr int ctrl = ((0 + K) & 3) | (((1 + K) & 3) << 2) | (((2 + K) & 3) << 4) | (((3 + K) & 3) << 6);
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)s, ctrl, 0xf, 0xf, false);
}

// The same encryption with one AES block per quad of lanes: lane c = lane % 4
// of the quad holds state column c (s) and computes output column c of every
// round, taking the bytes it needs from the other three columns by quad
// permutes.  A wave encrypts 16 blocks with 4 table lookups per lane and
// round, where aes_encrypt takes 16 per lane for up to 64 blocks, so it is the
// cheaper form for a tile's last 16 or fewer blocks.  The whole wave must be
// active.
__device__ __forceinline__ uint32_t aes_encrypt_quad(uint32_t s, uint32_t c, const AesLds &L) {
  const uint32_t *rk = L.rk;
  s ^= rk[c];
#pragma unroll
  for (int r = 1; r < 10; ++r) {
    const uint32_t n1 = quad_next<1>(s), n2 = quad_next<2>(s), n3 = quad_next<3>(s);
    s = xor3(xor3(L.t[0][s & 0xff], L.t[1][(n1 >> 8) & 0xff], L.t[2][(n2 >> 16) & 0xff]), L.t[3][n3 >> 24],
             rk[4 * r + c]);
  }
  const uint32_t n1 = quad_next<1>(s), n2 = quad_next<2>(s), n3 = quad_next<3>(s);
  const uint32_t t = (L.t[2][s & 0xff] & 0x000000ffu) | (L.t[3][(n1 >> 8) & 0xff] & 0x0000ff00u) |
                     (L.t[0][(n2 >> 16) & 0xff] & 0x00ff0000u) | (L.t[1][n3 >> 24] & 0xff000000u);
  return t ^ rk[40 + c];
}

// Counter block ctr0 + i (mod 2^128), big-endian; (hi, lo) are the numeric
// halves of ctr0.  Returns the four little-endian state words.
__device__ __forceinline__ void aes_counter(uint64_t hi, uint64_t lo, uint64_t i, uint32_t &w0, uint32_t &w1,
                                            uint32_t &w2, uint32_t &w3) {
  const uint64_t l = lo + i;
  const uint64_t h = hi + (l < lo ? 1u : 0u);
  w0 = __builtin_bswap32((uint32_t)(h >> 32));
  w1 = __builtin_bswap32((uint32_t)h);
  w2 = __builtin_bswap32((uint32_t)(l >> 32));
  w3 = __builtin_bswap32((uint32_t)l);
}

}  // namespace sf
