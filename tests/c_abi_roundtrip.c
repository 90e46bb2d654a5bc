/* A plain C consumer of the library: only include/sefrag.h and the HIP
 * runtime API, no Python.  Round-trips one deterministic 256 x 512 RGB image
 * (smooth ramps plus a hashed noise term) through the plain form (DC + 5 AC,
 * AES-CTR, exception slots), the fp16 precision form (residual codes), the
 * pixel-domain strong level and the wavelet form, and compares every sample; then takes the security statistics of
 * the image against its strong-level public part and compares their exact
 * integer fields with sums taken here on the host.  Prints one line per
 * form; exits non-zero on the first mismatch or error. */
#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "sefrag.h"

#define H 256
#define W 512
#define C 3

static int check(int rc, const char *what) {
  if (rc != SF_OK) {
    fprintf(stderr, "%s: %s (%s)\n", what, sf_strerror(rc), sf_last_error());
    exit(2);
  }
  return rc;
}

static void *dalloc(size_t n) {
  void *p = NULL;
  if (hipMalloc(&p, n ? n : 16) != hipSuccess) {
    fprintf(stderr, "hipMalloc(%zu) failed\n", n);
    exit(2);
  }
  return p;
}

static int compare(const uint8_t *d_out, const uint8_t *want, const char *form) {
  uint8_t *got = (uint8_t *)malloc((size_t)C * H * W);
  if (hipDeviceSynchronize() != hipSuccess || hipMemcpy(got, d_out, (size_t)C * H * W, hipMemcpyDeviceToHost) != hipSuccess) {
    fprintf(stderr, "%s: copy back failed\n", form);
    exit(2);
  }
  size_t bad = 0;
  for (size_t i = 0; i < (size_t)C * H * W; ++i) bad += got[i] != want[i];
  free(got);
  printf("%s: %zu of %d samples differ\n", form, bad, C * H * W);
  return bad == 0;
}

int main(void) {
  const size_t n = (size_t)C * H * W;
  uint8_t *img = (uint8_t *)malloc(n);
  for (int c = 0; c < C; ++c)
    for (int y = 0; y < H; ++y)
      for (int x = 0; x < W; ++x) {
        uint32_t h = (uint32_t)((c * H + y) * W + x) * 2654435761u;
        h ^= h >> 15;
        int v = 40 + (x * 150) / W + (y * 50) / H + c * 10 + (int)(h % 7u) - 3;
        img[((size_t)c * H + y) * W + x] = (uint8_t)(v < 0 ? 0 : v > 255 ? 255 : v);
      }
  check(sf_init(), "sf_init");
  uint8_t *d_img = (uint8_t *)dalloc(n), *d_out = (uint8_t *)dalloc(n);
  if (hipMemcpy(d_img, img, n, hipMemcpyHostToDevice) != hipSuccess) return 2;
  sf_aes_ctr aes;
  for (int i = 0; i < 16; ++i) {
    aes.key[i] = (uint8_t)(17 * i + 3);
    aes.ctr0[i] = i < 8 ? (uint8_t)(5 * i + 1) : 0;
  }
  int ok = 1;

  /* plain form */
  sf_desc d = {H, W, C, SF_FP32, (1ull << 6) - 1};
  size_t pb, qb, rb, eb;
  int needed;
  check(sf_fragment_sizes(&d, &pb, &qb, &rb), "sf_fragment_sizes");
  check(sf_exception_bytes(&d, 64, &eb, &needed), "sf_exception_bytes");
  void *d_pub = dalloc(pb);
  uint8_t *d_priv = (uint8_t *)dalloc(qb);
  sf_exceptions exc = {dalloc(eb), 64};
  uint32_t *d_status = (uint32_t *)dalloc(4);
  if (hipMemset(d_status, 0, 4) != hipSuccess) return 2;
  check(frag_image(&d, d_img, d_pub, d_priv, &exc, NULL, &aes, d_status, NULL), "frag_image");
  check(defrag_image(&d, d_pub, d_priv, &exc, NULL, &aes, d_out, d_status, NULL), "defrag_image");
  ok &= compare(d_out, img, "plain DC+5AC");
  uint32_t status = 1;
  if (hipMemcpy(&status, d_status, 4, hipMemcpyDeviceToHost) != hipSuccess || status != 0) {
    fprintf(stderr, "device status %u\n", status);
    ok = 0;
  }

  /* launch shapes: tune, read back, round trip in the tuned shapes, forget */
  {
    sf_launch_shape bf, bd, got;
    float fms = 0.0f, dms = 0.0f;
    check(sf_tune_image(&d, d_img, d_pub, d_priv, &exc, NULL, &aes, d_out, d_status, NULL, &bf, &bd, &fms, &dms),
          "sf_tune_image");
    ok &= compare(d_out, img, "plain DC+5AC, tuned shapes");
    check(sf_get_launch_shape(&d, 0, &got), "sf_get_launch_shape");
    if (got.waves_per_group != bf.waves_per_group || got.resident != bf.resident || !(fms > 0.0f) || !(dms > 0.0f)) {
      fprintf(stderr, "tuned shape not stored\n");
      ok = 0;
    }
    check(defrag_image(&d, d_pub, d_priv, &exc, NULL, &aes, d_out, d_status, NULL), "defrag_image tuned");
    ok &= compare(d_out, img, "plain DC+5AC, defrag in the tuned shape");
    check(sf_set_launch_shape(&d, 0, NULL), "sf_set_launch_shape");
    check(sf_set_launch_shape(&d, 1, NULL), "sf_set_launch_shape");
  }

  /* precision form: fp16 public values, 2-bit residual codes, exception slots */
  {
    sf_desc dl = d;
    dl.precision = SF_FP16;
    size_t lpb, lqb, lrb, leb;
    int lneeded = 0;
    check(sf_fragment_sizes(&dl, &lpb, &lqb, &lrb), "sf_fragment_sizes fp16");
    check(sf_exception_bytes(&dl, 16, &leb, &lneeded), "sf_exception_bytes fp16");
    if (lrb != (size_t)H * W * C / 4 || !lneeded) {
      fprintf(stderr, "fp16 sizes: residual %zu, exceptions needed %d\n", lrb, lneeded);
      ok = 0;
    }
    void *d_lpub = dalloc(lpb);
    uint8_t *d_lpriv = (uint8_t *)dalloc(lqb);
    int8_t *d_res = (int8_t *)dalloc(lrb);
    sf_exceptions lexc = {dalloc(leb), 16};
    check(frag_image(&dl, d_img, d_lpub, d_lpriv, &lexc, d_res, &aes, d_status, NULL), "frag_image fp16");
    check(defrag_image(&dl, d_lpub, d_lpriv, &lexc, d_res, &aes, d_out, d_status, NULL), "defrag_image fp16");
    ok &= compare(d_out, img, "precision fp16");
    hipFree(d_lpub);
    hipFree(d_lpriv);
    hipFree(d_res);
    hipFree(lexc.d_buf);
  }

  /* pixel-domain formats, strong level */
  size_t ppb, pqb;
  check(sf_pixel_fragment_sizes(&d, SF_LEVEL_STRONG, &ppb, &pqb), "sf_pixel_fragment_sizes");
  uint8_t *d_ppub = (uint8_t *)dalloc(ppb), *d_ppriv = (uint8_t *)dalloc(pqb);
  check(pixel_frag_image(&d, SF_LEVEL_STRONG, d_img, d_ppub, d_ppriv, &aes, NULL), "pixel_frag_image");
  check(pixel_defrag_image(&d, SF_LEVEL_STRONG, d_ppub, d_ppriv, &aes, d_out, NULL), "pixel_defrag_image");
  ok &= compare(d_out, img, "pixel strong");

  /* wavelet form */
  size_t wpb, wqb;
  check(sf_dwt_fragment_sizes(H, W, C, &wpb, &wqb), "sf_dwt_fragment_sizes");
  int16_t *d_wpub = (int16_t *)dalloc(wpb);
  uint8_t *d_wpriv = (uint8_t *)dalloc(wqb);
  check(dwt_frag_image(H, W, C, d_img, d_wpub, d_wpriv, &aes, NULL), "dwt_frag_image");
  check(dwt_defrag_image(H, W, C, d_wpub, d_wpriv, &aes, d_out, NULL), "dwt_defrag_image");
  ok &= compare(d_out, img, "wavelet");

  /* security statistics: image X against the strong-level public part Y */
  {
    const size_t wsb = sf_stats_workspace_bytes();
    void *d_ws = dalloc(wsb);
    sf_security_stats *d_st = (sf_security_stats *)dalloc(sizeof(sf_security_stats));
    check(sf_security_stats_compute(d_img, d_ppub, H, W, C, d_ws, wsb, d_st, NULL, NULL), "sf_security_stats_compute");
    sf_security_stats st;
    uint8_t *pub = (uint8_t *)malloc(n);
    if (hipDeviceSynchronize() != hipSuccess || hipMemcpy(&st, d_st, sizeof st, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(pub, d_ppub, n, hipMemcpyDeviceToHost) != hipSuccess) {
      fprintf(stderr, "statistics: copy back failed\n");
      exit(2);
    }
    uint64_t hx[256] = {0}, hy[256] = {0}, cross[6] = {n, 0, 0, 0, 0, 0}, pair[6] = {0}, bits = 0;
    for (size_t i = 0; i < n; ++i) {
      const uint64_t x = img[i], y = pub[i];
      ++hx[x];
      ++hy[y];
      cross[1] += x;
      cross[2] += y;
      cross[3] += x * x;
      cross[4] += y * y;
      cross[5] += x * y;
      bits += (uint64_t)__builtin_popcount((unsigned)(x ^ y));
    }
    /* horizontal pairs of X: (x, right neighbour) within each row of a plane */
    for (size_t r = 0; r < (size_t)C * H; ++r)
      for (int x = 0; x + 1 < W; ++x) {
        const uint64_t a = img[r * W + x], b = img[r * W + x + 1];
        ++pair[0];
        pair[1] += a;
        pair[2] += b;
        pair[3] += a * a;
        pair[4] += b * b;
        pair[5] += a * b;
      }
    size_t bad = 0;
    bad += st.samples != n;
    for (int v = 0; v < 256; ++v) bad += (st.hist_x[v] != hx[v]) + (st.hist_y[v] != hy[v]);
    for (int k = 0; k < 6; ++k) bad += (st.cross[k] != cross[k]) + (st.pair_x[0][k] != pair[k]);
    bad += st.bits_differing != bits;
    printf("statistics: %zu of %d exact fields differ\n", bad, 1 + 512 + 12 + 1);
    ok &= bad == 0;
    free(pub);
    hipFree(d_ws);
    hipFree(d_st);
  }

  /* a rejected call: height not a multiple of 8 */
  sf_desc bad = d;
  bad.height = 12;
  if (frag_image(&bad, d_img, d_pub, d_priv, &exc, NULL, &aes, d_status, NULL) != SF_ESHAPE) {
    fprintf(stderr, "bad shape not rejected\n");
    ok = 0;
  }

  hipFree(d_img); hipFree(d_out); hipFree(d_pub); hipFree(d_priv); hipFree(exc.d_buf); hipFree(d_status);
  hipFree(d_ppub); hipFree(d_ppriv); hipFree(d_wpub); hipFree(d_wpriv);
  free(img);
  printf(ok ? "c abi round trips ok\n" : "c abi round trips FAILED\n");
  return ok ? 0 : 1;
}
