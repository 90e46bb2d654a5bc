// Host generation of the library's constant tables, from their mathematical
// definitions:
//  * AES-128 S-box and round table (FIPS-197 Sec. 5.1.1: multiplicative
//    inverse in GF(2^8) followed by the affine map), key expansion (Sec. 5.2);
//  * 8-point DCT-II butterfly constants and the 64x64 orthonormal 8x8 DCT
//    basis (report Sec. 6.4.2: separable 2-D DCT), in long double;
//  * the integer basis round_half_even(2^20 B) of the private quantiser and
//    its signed-byte limbs;
//  * the integer basis round_half_even(2^16 B) of the pixel-domain inverse;
//  * per-coefficient bounds used by the exactness certificate.
#include <math.h>
#include <string.h>

#include <mutex>

#include "sf_internal.h"

namespace sf {
namespace {

// GF(2^8) with the AES polynomial x^8 + x^4 + x^3 + x + 1.
uint8_t gmul2(uint8_t a) { return (uint8_t)((a << 1) ^ ((a >> 7) * 0x1b)); }

void build_aes(HostTables &t) {
  // exp/log tables for the generator 3 (= x + 1)
  uint8_t ex[256], lg[256];
  uint8_t g = 1;
  for (int i = 0; i < 255; ++i) {
    ex[i] = g;
    lg[g] = (uint8_t)i;
    g = (uint8_t)(g ^ gmul2(g));  // g * 3
  }
  for (int x = 0; x < 256; ++x) {
    uint8_t inv = x == 0 ? 0 : ex[(255 - lg[x]) % 255];
    // affine map in rotation form: s = b ^ rotl1 ^ rotl2 ^ rotl3 ^ rotl4 ^ 0x63
    uint32_t b = inv;
    uint32_t s = b;
    for (int r = 1; r <= 4; ++r) s ^= ((b << r) | (b >> (8 - r))) & 0xff;
    t.sbox[x] = (uint8_t)(s ^ 0x63);
  }
  for (int x = 0; x < 256; ++x) {
    uint8_t s = t.sbox[x], s2 = gmul2(s), s3 = (uint8_t)(s2 ^ s);
    t.aes_t0[x] = (uint32_t)s2 | ((uint32_t)s << 8) | ((uint32_t)s << 16) | ((uint32_t)s3 << 24);
  }
}

long double dct_entry(int u, int i) {
  const long double pi = 3.141592653589793238462643383279502884L;
  long double c = u == 0 ? sqrtl(0.125L) : 0.5L;
  return c * cosl((2 * i + 1) * u * pi / 16.0L);
}

void build_dct(HostTables &t) {
  const long double pi = 3.141592653589793238462643383279502884L;
  t.dct.s0 = (float)sqrtl(0.125L);
  t.dct.a = (float)(0.5L * cosl(pi / 8.0L));
  t.dct.b = (float)(0.5L * cosl(3.0L * pi / 8.0L));
  t.dct.c1 = (float)(0.5L * cosl(pi / 16.0L));
  t.dct.c3 = (float)(0.5L * cosl(3.0L * pi / 16.0L));
  t.dct.c5 = (float)(0.5L * cosl(5.0L * pi / 16.0L));
  t.dct.c7 = (float)(0.5L * cosl(7.0L * pi / 16.0L));
  for (int u = 0; u < 8; ++u)
    for (int v = 0; v < 8; ++v) {
      const int n = 8 * u + v;
      long double maxabs = 0.0L, errsum = 0.0L;
      int64_t rowsum = 0;
      int32_t *qi = &t.q2_int[n * 64];
      for (int y = 0; y < 8; ++y)
        for (int x = 0; x < 8; ++x) {
          const long double bv = dct_entry(u, y) * dct_entry(v, x);
          t.basis[n * 64 + 8 * y + x] = (double)bv;
          const long double scaled = ldexpl(bv, 20);
          const int32_t q = (int32_t)llrintl(scaled);  // default rounding: to nearest, ties to even
          qi[8 * y + x] = q;
          t.inv16[n * 64 + 8 * y + x] = (int32_t)llrintl(ldexpl(bv, 16));
          rowsum += q;
          if (fabsl(bv) > maxabs) maxabs = fabsl(bv);
          errsum += fabsl((long double)q - scaled);
        }
      t.cert_m[n] = nextafterf((float)maxabs, 1.0f);
      t.cert_e[n] = nextafterf((float)(255.0L * ldexpl(errsum, -20)), 1.0f);
      // signed-byte limbs of every entry, 4 pixels per word
      uint32_t *row = &t.q2[n * kQ2RowWords];
      memset(row, 0, sizeof(uint32_t) * kQ2RowWords);
      for (int p = 0; p < 64; ++p) {
        int32_t q = qi[p];
        int32_t l = ((q + 128) & 0xff) - 128;
        int32_t rest = (q - l) / 256;
        int32_t m = ((rest + 128) & 0xff) - 128;
        int32_t h = (rest - m) / 256;
        const int w = p / 4, sh = 8 * (p % 4);
        row[w] |= (uint32_t)(uint8_t)(int8_t)l << sh;
        row[16 + w] |= (uint32_t)(uint8_t)(int8_t)m << sh;
        row[32 + w] |= (uint32_t)(uint8_t)(int8_t)h << sh;
      }
      row[48] = (uint32_t)(int32_t)(128 * rowsum);
      memcpy(&row[kQ2CertE], &t.cert_e[n], 4);
      memcpy(&row[kQ2CertM], &t.cert_m[n], 4);
    }
}

HostTables g_tables;
std::once_flag g_once;

}  // namespace

const HostTables &host_tables() {
  std::call_once(g_once, [] {
    build_aes(g_tables);
    build_dct(g_tables);
    build_lp_tables(g_tables.basis, g_tables.lp);
  });
  return g_tables;
}

// Floating-point allowance of the certificate: bounds the effect on any
// reconstructed sample of (a) the FP32 error of the stored public
// coefficients and (b) the FP32 evaluation error of the inverse transform.
// With u = 2^-24 and every butterfly output at most 6 roundings away from
// exact, per coefficient |dC| <= 2*8*255*6u*(1+6u) ~ 1.46e-3, so (a) <=
// 8 * 1.46e-3 (sum_n |B_n(p)| <= 8) and (b) <= 2*6u*sum_n |B_n(p)||c_n| <=
// 2.9e-3; 1/32 leaves a factor of two.  2^-12 covers the FP32 evaluation of
// the certificate sum itself.
float cert_threshold() { return 0.5f - 0x1p-5f - 0x1p-12f; }

bool mask_needs_check(uint64_t mask) {
  const HostTables &t = host_tables();
  static constexpr ZigZag zz{};
  double worst = 0.0;
  for (int z = 0; z < 64; ++z)
    if ((mask >> z) & 1u) {
      const int n = zz.nat[z];
      worst += (0.5 + (n == 0 ? 0.0 : (double)t.cert_e[n])) * (double)t.cert_m[n];
    }
  return worst >= (double)cert_threshold();
}

void aes_expand_key(const uint8_t key[16], uint32_t rk[44]) {
  const HostTables &t = host_tables();
  uint8_t w[176];
  memcpy(w, key, 16);
  uint8_t rcon = 1;
  for (int i = 16; i < 176; i += 4) {
    uint8_t tmp[4] = {w[i - 4], w[i - 3], w[i - 2], w[i - 1]};
    if (i % 16 == 0) {
      uint8_t f = tmp[0];
      tmp[0] = (uint8_t)(t.sbox[tmp[1]] ^ rcon);
      tmp[1] = t.sbox[tmp[2]];
      tmp[2] = t.sbox[tmp[3]];
      tmp[3] = t.sbox[f];
      rcon = gmul2(rcon);
    }
    for (int j = 0; j < 4; ++j) w[i + j] = (uint8_t)(w[i - 16 + j] ^ tmp[j]);
  }
  for (int i = 0; i < 44; ++i)
    rk[i] = (uint32_t)w[4 * i] | ((uint32_t)w[4 * i + 1] << 8) | ((uint32_t)w[4 * i + 2] << 16) |
            ((uint32_t)w[4 * i + 3] << 24);
}

}  // namespace sf
