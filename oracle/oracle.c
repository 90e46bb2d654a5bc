/*
 * Plain CPU oracle for DCT selective fragmentation -- TEST INFRASTRUCTURE ONLY.
 *
 * This file is the slow, obviously-correct reference against which the HIP
 * library is checked.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it.  It shares no code, header,
 * table or constant generator with the GPU library.
 *
 * What it computes (report "Data Protection: Combining Fragmentation,
 * Encryption, and Dispersion", Sec. 6.3.1 "First level of protection",
 * Fig. 6; Sec. 6.4.3 "Storage space and numeric precision"):
 *   - the 8x8 orthonormal DCT-II of every block of an 8-bit image (Sec. 6.1,
 *     Sec. 6.4.2), evaluated as a direct double sum in FP64;
 *   - the private fragment: DC plus the first k zigzag AC coefficients
 *     (default set [0,0],[0,1],[1,0],[2,0],[1,1],[0,2], Sec. 6.3.1), stored as
 *     integers (the 11-bit integer storage of Sec. 6.4.3, held in int16);
 *   - AES-128 (FIPS-197) in counter mode (NIST SP 800-38A) over the private
 *     byte stream (Sec. 6.5.2: AES on the selected part);
 *   - the public fragment: the remaining coefficients;
 *   - defragmentation (Sec. 5.2, Fig. 3): decrypt, merge, inverse DCT, round.
 *
 * Readings of points the report leaves open (all recorded in the design
 * notes): orthonormal DCT-II without level shift (DC bounded by 2040,
 * Sec. 6.4.3); JPEG zigzag order; integer quantiser "Q2" = round half to even
 * of sum_p x[p]*round(2^20*B[n][p]) / 2^20; int16 little endian; CTR counter is
 * the whole 128-bit block incremented big-endian; fragments in the 64-block
 * tile-interleaved layout described at orc_tile_offset().
 *
 * Parity status: every function here is pinned by the CPU test suite
 * (closed forms, library special cases, published AES/CTR vectors, brute
 * force); see the header comment of each function.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ */
/* 8x8 DCT-II basis (Sec. 6.1 / 6.4.2: separable 2-D DCT on 8x8 blocks). */
/* B[n][p], n = 8u+v (u vertical frequency, v horizontal), p = 8y+x.     */
/*   B[n][p] = c(u) c(v) cos((2y+1)u pi/16) cos((2x+1)v pi/16)           */
/*   c(0) = sqrt(1/8), c(u>0) = sqrt(2/8) = 1/2  (orthonormal).          */
/* Pinned by: B B^T = I, DC row = 1/8, scipy dctn(norm='ortho').          */
/* ------------------------------------------------------------------ */
void orc_basis(double *B) {
  const double pi = acos(-1.0);
  for (int u = 0; u < 8; ++u)
    for (int v = 0; v < 8; ++v)
      for (int y = 0; y < 8; ++y)
        for (int x = 0; x < 8; ++x) {
          double cu = (u == 0) ? sqrt(1.0 / 8.0) : sqrt(2.0 / 8.0);
          double cv = (v == 0) ? sqrt(1.0 / 8.0) : sqrt(2.0 / 8.0);
          B[(8 * u + v) * 64 + (8 * y + x)] =
              cu * cv * cos((2 * y + 1) * u * pi / 16.0) * cos((2 * x + 1) * v * pi / 16.0);
        }
}

/* ------------------------------------------------------------------ */
/* Zigzag order: walk the anti-diagonals u+v = s, s = 0..14; on odd s the  */
/* row index u increases, on even s it decreases (JPEG order).  zz[z] is   */
/* the natural index 8u+v of zigzag position z.  Pinned by the default     */
/* private list of Sec. 6.3.1: [0,0],[0,1],[1,0],[2,0],[1,1],[0,2].        */
/* ------------------------------------------------------------------ */
void orc_zigzag(int *zz) {
  int z = 0;
  for (int s = 0; s <= 14; ++s) {
    if (s % 2 == 1) {
      for (int u = 0; u <= 7; ++u) {
        int v = s - u;
        if (v >= 0 && v <= 7) zz[z++] = 8 * u + v;
      }
    } else {
      for (int u = 7; u >= 0; --u) {
        int v = s - u;
        if (v >= 0 && v <= 7) zz[z++] = 8 * u + v;
      }
    }
  }
}

/* Integer basis for the private quantiser: Bq[n][p] = round_half_even(2^20 B[n][p]).
 * Pinned against a 50-digit mpmath rebuild of the same table. */
void orc_q2_table(int32_t *Bq) {
  double B[64 * 64];
  orc_basis(B);
  for (int i = 0; i < 64 * 64; ++i) Bq[i] = (int32_t)nearbyint(ldexp(B[i], 20));
}

/* Round half to even of acc / 2^20, written out with an explicit floor
 * division and remainder (reading of "quantised to integers", Sec. 6.4.3). */
static int32_t orc_round_q20(int64_t acc) {
  const int64_t one = (int64_t)1 << 20, half = (int64_t)1 << 19;
  int64_t m = acc / one;                 /* truncates toward zero */
  if (acc % one != 0 && acc < 0) m -= 1; /* make it a floor */
  int64_t r = acc - m * one;             /* 0 <= r < 2^20 */
  if (r > half) m += 1;
  else if (r == half && (m % 2 != 0)) m += 1;
  return (int32_t)m;
}

/* ------------------------------------------------------------------ */
/* Block addressing.  Planes c = 0..C-1 of H x W bytes, row-major, planar. */
/* Block b = (c*By + by)*Bx + bx, By = H/8, Bx = W/8.                     */
/* ------------------------------------------------------------------ */
static void orc_load_block(const uint8_t *pix, int H, int W, int64_t b, double *xb, int32_t *xi) {
  int64_t Bx = W / 8, By = H / 8;
  int64_t c = b / (Bx * By), rem = b % (Bx * By);
  int64_t by = rem / Bx, bx = rem % Bx;
  const uint8_t *base = pix + c * (int64_t)H * W + (by * 8) * (int64_t)W + bx * 8;
  for (int y = 0; y < 8; ++y)
    for (int x = 0; x < 8; ++x) {
      uint8_t v = base[(int64_t)y * W + x];
      if (xb) xb[8 * y + x] = (double)v;
      if (xi) xi[8 * y + x] = (int32_t)v;
    }
}
static int64_t orc_pixel_index(int H, int W, int64_t b, int p) {
  int64_t Bx = W / 8, By = H / 8;
  int64_t c = b / (Bx * By), rem = b % (Bx * By);
  int64_t by = rem / Bx, bx = rem % Bx;
  return c * (int64_t)H * W + (by * 8 + p / 8) * (int64_t)W + bx * 8 + p % 8;
}

/* Tile-interleaved fragment layout: blocks are grouped in tiles of 64
 * consecutive block indices; tile t holds n_t = min(64, nb - 64t) blocks and
 * stores value j of its block i (0 <= i < n_t) at element
 *   64*t*P + j*n_t + i,        P = values per block.
 * The layout is dense (no padding) for any block count. */
int64_t orc_tile_offset(int64_t nb, int64_t P, int64_t b, int64_t j) {
  int64_t t = b / 64, i = b % 64;
  int64_t nt = nb - 64 * t;
  if (nt > 64) nt = 64;
  return 64 * t * P + j * nt + i;
}

/* Direct FP64 DCT of every block: coef[b*64 + n]. */
void orc_dct_blocks(const uint8_t *pix, int C, int H, int W, double *coef) {
  double B[64 * 64];
  orc_basis(B);
  int64_t nb = (int64_t)C * (H / 8) * (W / 8);
#pragma omp parallel for schedule(static)
  for (int64_t b = 0; b < nb; ++b) {
    double xb[64];
    orc_load_block(pix, H, W, b, xb, NULL);
    for (int n = 0; n < 64; ++n) {
      double s = 0.0;
      for (int p = 0; p < 64; ++p) s += B[n * 64 + p] * xb[p];
      coef[b * 64 + n] = s;
    }
  }
}

/* Direct FP64 inverse DCT: y[b*64 + p] = sum_n B[n][p] coef[b*64+n]. */
void orc_idct_blocks(const double *coef, int64_t nb, double *y) {
  double B[64 * 64];
  orc_basis(B);
#pragma omp parallel for schedule(static)
  for (int64_t b = 0; b < nb; ++b)
    for (int p = 0; p < 64; ++p) {
      double s = 0.0;
      for (int n = 0; n < 64; ++n) s += B[n * 64 + p] * coef[b * 64 + n];
      y[b * 64 + p] = s;
    }
}

/* Q2 private quantiser for a list of natural indices: q[b*nl + l]. */
void orc_q2_blocks(const uint8_t *pix, int C, int H, int W, const int *nat, int nl, int32_t *q) {
  int32_t Bq[64 * 64];
  orc_q2_table(Bq);
  int64_t nb = (int64_t)C * (H / 8) * (W / 8);
#pragma omp parallel for schedule(static)
  for (int64_t b = 0; b < nb; ++b) {
    int32_t xi[64];
    orc_load_block(pix, H, W, b, NULL, xi);
    for (int l = 0; l < nl; ++l) {
      int64_t acc = 0;
      for (int p = 0; p < 64; ++p) acc += (int64_t)xi[p] * Bq[nat[l] * 64 + p];
      q[b * nl + l] = orc_round_q20(acc);
    }
  }
}

/* ------------------------------------------------------------------ */
/* AES-128, FIPS-197.  Byte-oriented textbook form.                        */
/* Pinned by the FIPS-197 Appendix B / C.1 examples and by openssl.        */
/* ------------------------------------------------------------------ */
static uint8_t gf_xtime(uint8_t a) { return (uint8_t)((a << 1) ^ ((a & 0x80) ? 0x1b : 0x00)); }
static uint8_t gf_mul(uint8_t a, uint8_t b) {
  uint8_t p = 0;
  while (b) {
    if (b & 1) p ^= a;
    a = gf_xtime(a);
    b >>= 1;
  }
  return p;
}
/* Multiplicative inverse in GF(2^8) (0 maps to 0): a^254. */
static uint8_t gf_inv(uint8_t a) {
  uint8_t r = 1;
  for (int i = 0; i < 254; ++i) r = gf_mul(r, a);
  return a ? r : 0;
}
/* S-box (FIPS-197 Sec. 5.1.1): inverse, then the affine map
 * b'_i = b_i ^ b_{i+4} ^ b_{i+5} ^ b_{i+6} ^ b_{i+7} ^ c_i, c = 0x63. */
void orc_aes_sbox(uint8_t *sbox) {
  for (int a = 0; a < 256; ++a) {
    uint8_t b = gf_inv((uint8_t)a), s = 0;
    for (int i = 0; i < 8; ++i) {
      int bit = ((b >> i) ^ (b >> ((i + 4) % 8)) ^ (b >> ((i + 5) % 8)) ^ (b >> ((i + 6) % 8)) ^
                 (b >> ((i + 7) % 8)) ^ (0x63 >> i)) & 1;
      s |= (uint8_t)(bit << i);
    }
    sbox[a] = s;
  }
}
/* Key expansion (FIPS-197 Sec. 5.2), Nk = 4, Nr = 10: 176 bytes. */
void orc_aes_expand(const uint8_t key[16], uint8_t rk[176]) {
  uint8_t sbox[256];
  orc_aes_sbox(sbox);
  memcpy(rk, key, 16);
  uint8_t rcon = 1;
  for (int i = 4; i < 44; ++i) {
    uint8_t t[4];
    memcpy(t, rk + 4 * (i - 1), 4);
    if (i % 4 == 0) {
      uint8_t t0 = t[0];
      t[0] = (uint8_t)(sbox[t[1]] ^ rcon);
      t[1] = sbox[t[2]];
      t[2] = sbox[t[3]];
      t[3] = sbox[t0];
      rcon = gf_xtime(rcon);
    }
    for (int j = 0; j < 4; ++j) rk[4 * i + j] = (uint8_t)(rk[4 * (i - 4) + j] ^ t[j]);
  }
}
/* Cipher (FIPS-197 Sec. 5.1).  State s[r + 4c] = in[r + 4c] (column-major). */
static void orc_aes_encrypt_rk(const uint8_t rk[176], const uint8_t *sbox, const uint8_t in[16], uint8_t out[16]) {
  uint8_t s[16], t[16];
  for (int i = 0; i < 16; ++i) s[i] = (uint8_t)(in[i] ^ rk[i]);
  for (int round = 1; round <= 10; ++round) {
    for (int i = 0; i < 16; ++i) s[i] = sbox[s[i]];                 /* SubBytes */
    for (int r = 0; r < 4; ++r)                                     /* ShiftRows */
      for (int c = 0; c < 4; ++c) t[r + 4 * c] = s[r + 4 * ((c + r) % 4)];
    if (round != 10) {                                              /* MixColumns */
      for (int c = 0; c < 4; ++c) {
        uint8_t a0 = t[4 * c], a1 = t[4 * c + 1], a2 = t[4 * c + 2], a3 = t[4 * c + 3];
        s[4 * c + 0] = (uint8_t)(gf_mul(a0, 2) ^ gf_mul(a1, 3) ^ a2 ^ a3);
        s[4 * c + 1] = (uint8_t)(a0 ^ gf_mul(a1, 2) ^ gf_mul(a2, 3) ^ a3);
        s[4 * c + 2] = (uint8_t)(a0 ^ a1 ^ gf_mul(a2, 2) ^ gf_mul(a3, 3));
        s[4 * c + 3] = (uint8_t)(gf_mul(a0, 3) ^ a1 ^ a2 ^ gf_mul(a3, 2));
      }
    } else {
      memcpy(s, t, 16);
    }
    for (int i = 0; i < 16; ++i) s[i] ^= rk[16 * round + i];       /* AddRoundKey */
  }
  memcpy(out, s, 16);
}
void orc_aes128_encrypt(const uint8_t key[16], const uint8_t in[16], uint8_t out[16]) {
  uint8_t rk[176], sbox[256];
  orc_aes_expand(key, rk);
  orc_aes_sbox(sbox);
  orc_aes_encrypt_rk(rk, sbox, in, out);
}

/* CTR mode (SP 800-38A Sec. 6.5, counter blocks T_i = ctr0 + i mod 2^128,
 * big-endian over all 16 bytes).  out[j] = in[j] ^ E_K(T_{first + j/16})[j%16].
 * A trailing partial block uses the leading bytes of its keystream block. */
static void orc_ctr_block(const uint8_t ctr0[16], uint64_t i, uint8_t T[16]) {
  unsigned carry = 0;
  uint64_t add = i;
  for (int byte = 15; byte >= 0; --byte) {
    unsigned v = ctr0[byte] + (unsigned)(add & 0xff) + carry;
    T[byte] = (uint8_t)(v & 0xff);
    carry = v >> 8;
    add >>= 8;
  }
}
void orc_ctr_xor(const uint8_t key[16], const uint8_t ctr0[16], uint64_t first_block,
                 const uint8_t *in, uint8_t *out, int64_t nbytes) {
  uint8_t rk[176], sbox[256];
  orc_aes_expand(key, rk);
  orc_aes_sbox(sbox);
  int64_t nblk = (nbytes + 15) / 16;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < nblk; ++i) {
    uint8_t T[16], ks[16];
    orc_ctr_block(ctr0, first_block + (uint64_t)i, T);
    orc_aes_encrypt_rk(rk, sbox, T, ks);
    for (int j = 0; j < 16 && 16 * i + j < nbytes; ++j) out[16 * i + j] = (uint8_t)(in[16 * i + j] ^ ks[j]);
  }
}

/* ------------------------------------------------------------------ */
/* Whole first-level-of-protection pipeline (Sec. 6.3.1, Fig. 6).          */
/* ------------------------------------------------------------------ */
static int orc_popcount64(uint64_t m) {
  int c = 0;
  while (m) {
    c += (int)(m & 1);
    m >>= 1;
  }
  return c;
}

/* Fragmentation.
 *   mask  : bit z set <=> zigzag position z is private.
 *   pub   : nb*(64-|mask|) doubles, tile layout, zigzag order (FP64 public).
 *   priv  : nb*|mask| int16, tile layout, zigzag order (plaintext).
 *   cipher: 2*nb*|mask| bytes, AES-CTR of the little-endian priv bytes, or
 *           NULL (then key/ctr0 unused).
 *   exc_index/exc_value/exc_cap: pixels whose FP64 reconstruction from the
 *           stored fragments does not round back to the input, in block
 *           order; returns their count (may exceed exc_cap), or -1 when a
 *           private integer does not fit int16.
 *   max_err: largest |IDCT(stored) - x| over all pixels (FP64). */
int64_t orc_frag(const uint8_t *pix, int C, int H, int W, uint64_t mask, double *pub, int16_t *priv,
                 const uint8_t *key, const uint8_t *ctr0, uint8_t *cipher, int64_t *exc_index,
                 uint8_t *exc_value, int64_t exc_cap, double *max_err) {
  int zz[64];
  double B[64 * 64];
  int32_t Bq[64 * 64];
  orc_zigzag(zz);
  orc_basis(B);
  orc_q2_table(Bq);
  const int npriv = orc_popcount64(mask), npub = 64 - npriv;
  const int64_t nb = (int64_t)C * (H / 8) * (W / 8);
  uint8_t *miss = (uint8_t *)calloc((size_t)(nb > 0 ? nb : 1), 64);
  int64_t bad = 0, nexc = 0;
  double worst = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : bad) reduction(max : worst)
  for (int64_t b = 0; b < nb; ++b) {
    double xb[64], coef[64], stored[64];
    int32_t xi[64];
    orc_load_block(pix, H, W, b, xb, xi);
    for (int n = 0; n < 64; ++n) {
      double s = 0.0;
      for (int p = 0; p < 64; ++p) s += B[n * 64 + p] * xb[p];
      coef[n] = s;
    }
    int jpriv = 0, jpub = 0;
    for (int z = 0; z < 64; ++z) {
      int n = zz[z];
      if ((mask >> z) & 1) {
        int64_t acc = 0;
        for (int p = 0; p < 64; ++p) acc += (int64_t)xi[p] * Bq[n * 64 + p];
        int32_t q = orc_round_q20(acc);
        if (q < -32768 || q > 32767) bad += 1;
        priv[orc_tile_offset(nb, npriv, b, jpriv++)] = (int16_t)q;
        stored[n] = (double)q;
      } else {
        pub[orc_tile_offset(nb, npub, b, jpub++)] = coef[n];
        stored[n] = coef[n];
      }
    }
    /* reconstruction from the stored values (Sec. 6.4.3: lossless or not) */
    for (int p = 0; p < 64; ++p) {
      double y = 0.0;
      for (int n = 0; n < 64; ++n) y += B[n * 64 + p] * stored[n];
      double e = fabs(y - xb[p]);
      if (e > worst) worst = e;
      double r = nearbyint(y);
      if (r < 0) r = 0;
      if (r > 255) r = 255;
      if (r != xb[p]) miss[b * 64 + p] = 1;
    }
  }
  if (max_err) *max_err = worst;
  if (bad) {
    free(miss);
    return -1;
  }
  for (int64_t b = 0; b < nb; ++b)
    for (int p = 0; p < 64; ++p)
      if (miss[b * 64 + p]) {
        if (nexc < exc_cap) {
          int64_t idx = orc_pixel_index(H, W, b, p);
          exc_index[nexc] = idx;
          exc_value[nexc] = pix[idx];
        }
        nexc++;
      }
  free(miss);
  if (cipher) {
    int64_t nbytes = 2 * nb * npriv;
    uint8_t *plain = (uint8_t *)malloc((size_t)(nbytes > 0 ? nbytes : 1));
    for (int64_t i = 0; i < nb * npriv; ++i) {
      uint16_t u = (uint16_t)priv[i];
      plain[2 * i] = (uint8_t)(u & 0xff);
      plain[2 * i + 1] = (uint8_t)(u >> 8);
    }
    orc_ctr_xor(key, ctr0, 0, plain, cipher, nbytes);
    free(plain);
  }
  return nexc;
}

/* Defragmentation (Sec. 5.2, Fig. 3): decrypt (if cipher given), merge the
 * private integers and public coefficients in zigzag order, FP64 inverse DCT,
 * round half to even, clamp to [0,255], then apply the exception list. */
void orc_defrag(int C, int H, int W, uint64_t mask, const double *pub, const int16_t *priv,
                const uint8_t *key, const uint8_t *ctr0, const uint8_t *cipher, const int64_t *exc_index,
                const uint8_t *exc_value, int64_t nexc, uint8_t *out) {
  int zz[64];
  double B[64 * 64];
  orc_zigzag(zz);
  orc_basis(B);
  const int npriv = orc_popcount64(mask), npub = 64 - npriv;
  const int64_t nb = (int64_t)C * (H / 8) * (W / 8);
  int16_t *q = (int16_t *)malloc((size_t)(nb * npriv > 0 ? nb * npriv : 1) * sizeof(int16_t));
  if (cipher) {
    int64_t nbytes = 2 * nb * npriv;
    uint8_t *plain = (uint8_t *)malloc((size_t)(nbytes > 0 ? nbytes : 1));
    orc_ctr_xor(key, ctr0, 0, cipher, plain, nbytes);
    for (int64_t i = 0; i < nb * npriv; ++i) q[i] = (int16_t)(uint16_t)(plain[2 * i] | (plain[2 * i + 1] << 8));
    free(plain);
  } else {
    memcpy(q, priv, (size_t)(nb * npriv) * sizeof(int16_t));
  }
#pragma omp parallel for schedule(static)
  for (int64_t b = 0; b < nb; ++b) {
    double stored[64];
    int jpriv = 0, jpub = 0;
    for (int z = 0; z < 64; ++z) {
      int n = zz[z];
      if ((mask >> z) & 1) stored[n] = (double)q[orc_tile_offset(nb, npriv, b, jpriv++)];
      else stored[n] = pub[orc_tile_offset(nb, npub, b, jpub++)];
    }
    for (int p = 0; p < 64; ++p) {
      double y = 0.0;
      for (int n = 0; n < 64; ++n) y += B[n * 64 + p] * stored[n];
      double r = nearbyint(y);
      if (r < 0) r = 0;
      if (r > 255) r = 255;
      out[orc_pixel_index(H, W, b, p)] = (uint8_t)r;
    }
  }
  for (int64_t e = 0; e < nexc; ++e) out[exc_index[e]] = exc_value[e];
  free(q);
}

void orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}
int orc_get_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Keystream blocks E_K(ctr0 + idx[i]) for a list of block indices (CTR
 * definition of SP 800-38A, as orc_ctr_xor); out holds 16 bytes per index. */
void orc_ctr_keystream(const uint8_t key[16], const uint8_t ctr0[16], const uint64_t *idx, int64_t n, uint8_t *out) {
  uint8_t rk[176], sbox[256];
  orc_aes_expand(key, rk);
  orc_aes_sbox(sbox);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    uint8_t T[16];
    orc_ctr_block(ctr0, idx[i], T);
    orc_aes_encrypt_rk(rk, sbox, T, out + 16 * i);
  }
}
