// C ABI entry points: validation, lazy per-device initialisation, dispatch.
#include <string.h>

#include <mutex>
#include <string>

#include "sf_internal.h"

namespace sf {

static thread_local std::string t_last_error;

int fail(int code, const std::string &msg) {
  t_last_error = msg;
  return code;
}

int hip_fail(hipError_t e, const char *what) {
  t_last_error = std::string(what) + ": " + hipGetErrorString(e);
  return SF_EHIP;
}

int make_geom(const sf_desc *d, Geom *g) {
  if (!d) return fail(SF_EINVAL, "desc is NULL");
  if (d->height == 0 || d->width == 0 || d->height % 8 || d->width % 8)
    return fail(SF_ESHAPE, "height and width must be positive multiples of 8");
  if (d->channels == 0) return fail(SF_ESHAPE, "channels must be >= 1");
  const uint64_t samples = (uint64_t)d->height * d->width * d->channels;
  if (samples >= (1ull << 32)) return fail(SF_ESHAPE, "image must hold fewer than 2^32 samples");
  if (d->precision > SF_BF16) return fail(SF_EINVAL, "unknown precision");
  if (d->private_mask == 0) return fail(SF_EINVAL, "private_mask must select at least one coefficient");
  g->H = d->height;
  g->W = d->width;
  g->C = d->channels;
  g->Bx = d->width / 8;
  g->By = d->height / 8;
  g->nb = samples / 64;
  g->ntiles = (uint32_t)((g->nb + 63) / 64);
  g->mask = d->private_mask;
  g->npriv = (uint32_t)__builtin_popcountll(d->private_mask);
  g->npub = 64 - g->npriv;
  g->precision = d->precision;
  return SF_OK;
}

// Kernels read 8-byte pixel rows and 16-byte private chunks.
static int check_alignment(const void *pix, const void *pub, const void *priv) {
  if ((uintptr_t)pix & 7u) return fail(SF_EINVAL, "pixel buffer must be 8-byte aligned");
  if ((uintptr_t)pub & 15u) return fail(SF_EINVAL, "public fragment must be 16-byte aligned");
  if ((uintptr_t)priv & 15u) return fail(SF_EINVAL, "private fragment must be 16-byte aligned");
  return SF_OK;
}

static size_t align16(size_t v) { return (v + 15u) & ~(size_t)15u; }

ExcLayout exc_layout(const Geom &g, uint32_t per_tile) {
  ExcLayout L;
  L.pos_offset = align16((size_t)2 * g.ntiles);
  L.val_offset = L.pos_offset + align16((size_t)2 * g.ntiles * per_tile);
  L.total = L.val_offset + align16((size_t)g.ntiles * per_tile);
  return L;
}

void make_aes_args(const sf_aes_ctr *aes, AesArgs *a) {
  memset(a, 0, sizeof(*a));
  if (!aes) return;
  a->enabled = 1;
  aes_expand_key(aes->key, a->key.rk);
  uint64_t hi = 0, lo = 0;
  for (int i = 0; i < 8; ++i) hi = (hi << 8) | aes->ctr0[i];
  for (int i = 8; i < 16; ++i) lo = (lo << 8) | aes->ctr0[i];
  a->ctr_hi = hi;
  a->ctr_lo = lo;
}

static std::mutex g_dev_mu;
static DeviceState g_dev[64];

int device_state(DeviceState **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= 64) return fail(SF_ENOTSUP, "device index out of range");
  std::lock_guard<std::mutex> lk(g_dev_mu);
  DeviceState &s = g_dev[dev];
  if (s.device < 0) {
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
      return fail(SF_ENOTSUP, std::string("library is built for gfx950, device is ") + prop.gcnArchName);
    const HostTables &t = host_tables();
    uint32_t *d_t0 = nullptr, *d_q2 = nullptr, *d_lp = nullptr;
    auto release = [&] {
      if (d_t0) (void)hipFree(d_t0);
      if (d_q2) (void)hipFree(d_q2);
      if (d_lp) (void)hipFree(d_lp);
    };
    if ((e = hipMalloc(&d_t0, sizeof(t.aes_t0))) != hipSuccess || (e = hipMalloc(&d_q2, sizeof(t.q2))) != hipSuccess ||
        (e = hipMalloc(&d_lp, sizeof(t.lp))) != hipSuccess) {
      release();
      return hip_fail(e, "hipMalloc(tables)");
    }
    if ((e = hipMemcpy(d_t0, t.aes_t0, sizeof(t.aes_t0), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(d_q2, t.q2, sizeof(t.q2), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(d_lp, t.lp, sizeof(t.lp), hipMemcpyHostToDevice)) != hipSuccess) {
      release();
      return hip_fail(e, "hipMemcpy(tables)");
    }
    // the allocation-free soft-mask forward's scratch array, at its address
    // on this device (the current one)
    void *sm_scratch = nullptr;
    if (int rc = softmask_scratch_address(&sm_scratch)) {
      release();
      return rc;
    }
    s.d_sm_scratch = sm_scratch;
    s.num_cu = prop.multiProcessorCount;
    s.max_lds_per_block = prop.sharedMemPerBlock;
    s.d_aes_t0 = d_t0;
    s.d_q2 = d_q2;
    s.d_lp = d_lp;
    s.device = dev;
  }
  *out = &s;
  return SF_OK;
}

// Size class of an image: ceil(log2(number of tiles)).
static uint32_t size_class(const Geom &g) {
  uint32_t c = 0;
  while (c < 32 && (1ull << c) < g.ntiles) ++c;
  return c;
}

static ShapeKey shape_key(const Geom &g, int which) { return ShapeKey(g.precision, g.mask, size_class(g), which); }

Shape stored_shape(DeviceState &ds, const Geom &g, int which) {
  std::lock_guard<std::mutex> lk(ds.shape_mu);
  auto it = ds.shapes.find(shape_key(g, which));
  if (it != ds.shapes.end()) return it->second;
  // plain form: one tile per wave, except defrag of 8 or more private
  // coefficients (resident); reduced precision: resident
  return Shape{0u, g.precision == SF_FP32 && !(plain_heavy(g) && which == 1) ? 0u : 1u};
}

// The shape a launch of (g, which) would use, resolved (waves >= 1).
static int resolved_shape(const DeviceState &ds, const Geom &g, int which, const Shape &in, Shape *out) {
  *out = in;
  if (g.precision == SF_FP32) {
    if (!out->waves) out->waves = plain_default_waves(g, which);
    return plain_lds_bytes(g, which, out->waves) <= ds.max_lds_per_block
               ? SF_OK
               : fail(SF_ENOTSUP, "launch shape: the workgroup's LDS does not fit on this device");
  }
  if (!out->waves) out->waves = lp_default_waves(ds, g, which);
  if (!out->waves || lp_lds_bytes(g, which, out->waves) > ds.max_lds_per_block)
    return fail(SF_ENOTSUP, "launch shape: the workgroup's LDS does not fit on this device");
  return SF_OK;
}

}  // namespace sf

using namespace sf;

extern "C" {

const char *sf_version(void) { return "sefrag 0.1 (gfx950)"; }

const char *sf_strerror(int code) {
  switch (code) {
    case SF_OK: return "ok";
    case SF_EINVAL: return "invalid argument";
    case SF_ESHAPE: return "invalid image shape";
    case SF_ERANGE: return "size or capacity out of range";
    case SF_EHIP: return "HIP runtime error";
    case SF_ENOTSUP: return "not supported";
    default: return "unknown error";
  }
}

const char *sf_last_error(void) { return t_last_error.c_str(); }

int sf_fragment_sizes(const sf_desc *desc, size_t *public_bytes, size_t *private_bytes, size_t *residual_bytes) {
  Geom g;
  int rc = make_geom(desc, &g);
  if (rc) return rc;
  const size_t elt = g.precision == SF_FP32 ? 4 : 2;
  if (public_bytes) *public_bytes = (size_t)g.nb * g.npub * elt;
  if (private_bytes) *private_bytes = (size_t)g.nb * g.npriv * 2;
  if (residual_bytes) *residual_bytes = g.precision == SF_FP32 ? 0 : (size_t)g.nb * 16;
  t_last_error.clear();
  return SF_OK;
}

int sf_exception_bytes(const sf_desc *desc, uint32_t per_tile, size_t *bytes, int *needed) {
  Geom g;
  int rc = make_geom(desc, &g);
  if (rc) return rc;
  if (per_tile > kMaxExcPerTile) return fail(SF_ERANGE, "per_tile must be at most 4096");
  if (bytes) *bytes = exc_layout(g, per_tile).total;
  if (needed) *needed = (g.precision != SF_FP32 || mask_needs_check(g.mask)) ? 1 : 0;
  t_last_error.clear();
  return SF_OK;
}

int sf_init(void) {
  DeviceState *ds;
  return device_state(&ds);
}

// Checks shared by frag_image and defrag_image.
static int check_call(const Geom &g, const void *pix, const void *pub, const void *priv, const sf_exceptions *exc,
                      const void *residual) {
  if (!pix || !priv || (g.npub && !pub)) return fail(SF_EINVAL, "NULL fragment or image pointer");
  int rc = check_alignment(pix, pub, priv);
  if (rc) return rc;
  if (g.precision != SF_FP32 || mask_needs_check(g.mask)) {
    if (!exc || !exc->d_buf) return fail(SF_EINVAL, "this selection needs an exception buffer");
    if (exc->per_tile == 0 || exc->per_tile > kMaxExcPerTile)
      return fail(SF_ERANGE, "exception slots per tile must be 1 .. 4096");
    if ((uintptr_t)exc->d_buf & 15u) return fail(SF_EINVAL, "exception buffer must be 16-byte aligned");
  }
  if (g.precision != SF_FP32) {
    if (!residual) return fail(SF_EINVAL, "reduced-precision forms need a residual code buffer");
    if ((uintptr_t)residual & 15u) return fail(SF_EINVAL, "residual code buffer must be 16-byte aligned");
  }
  return SF_OK;
}

int frag_image(const sf_desc *desc, const uint8_t *d_pixels, void *d_public, uint8_t *d_private,
               const sf_exceptions *exc, int8_t *d_residual, const sf_aes_ctr *aes, uint32_t *d_status,
               void *stream) {
  Geom g;
  int rc = make_geom(desc, &g);
  if (rc) return rc;
  if ((rc = check_call(g, d_pixels, d_public, d_private, exc, d_residual))) return rc;
  DeviceState *ds;
  if ((rc = device_state(&ds))) return rc;
  AesArgs a;
  make_aes_args(aes, &a);
  const Shape sh = stored_shape(*ds, g, 0);
  if (g.precision == SF_FP32)
    rc = launch_frag_fp32(*ds, g, d_pixels, (float *)d_public, d_private, exc, a, d_status, sh, (hipStream_t)stream);
  else
    rc = launch_frag_lp(*ds, g, d_pixels, d_public, d_private, exc, (uint8_t *)d_residual, a, d_status, sh,
                        (hipStream_t)stream);
  if (rc == SF_OK) t_last_error.clear();
  return rc;
}

int defrag_image(const sf_desc *desc, const void *d_public, const uint8_t *d_private, const sf_exceptions *exc,
                 const int8_t *d_residual, const sf_aes_ctr *aes, uint8_t *d_pixels, uint32_t *d_status,
                 void *stream) {
  Geom g;
  int rc = make_geom(desc, &g);
  if (rc) return rc;
  if ((rc = check_call(g, d_pixels, d_public, d_private, exc, d_residual))) return rc;
  DeviceState *ds;
  if ((rc = device_state(&ds))) return rc;
  AesArgs a;
  make_aes_args(aes, &a);
  const Shape sh = stored_shape(*ds, g, 1);
  if (g.precision == SF_FP32)
    rc = launch_defrag_fp32(*ds, g, (const float *)d_public, d_private, exc, a, d_pixels, sh, (hipStream_t)stream);
  else
    rc = launch_defrag_lp(*ds, g, d_public, d_private, exc, (const uint8_t *)d_residual, a, d_pixels, d_status, sh,
                          (hipStream_t)stream);
  if (rc == SF_OK) t_last_error.clear();
  return rc;
}

static bool valid_shape(const sf_launch_shape *s) {
  const uint32_t w = s->waves_per_group;
  return (w == 0 || w == 1 || w == 2 || w == 4 || w == 6 || w == 8) && s->resident <= 1;
}

int sf_set_launch_shape(const sf_desc *desc, int which, const sf_launch_shape *shape) {
  Geom g;
  int rc = make_geom(desc, &g);
  if (rc) return rc;
  if (which != 0 && which != 1) return fail(SF_EINVAL, "which must be 0 (frag) or 1 (defrag)");
  if (shape && !valid_shape(shape)) return fail(SF_EINVAL, "waves_per_group must be 0, 1, 2, 4, 6 or 8; resident 0 or 1");
  DeviceState *ds;
  if ((rc = device_state(&ds))) return rc;
  if (shape) {
    Shape r;
    if ((rc = resolved_shape(*ds, g, which, Shape{shape->waves_per_group, shape->resident}, &r))) return rc;
    std::lock_guard<std::mutex> lk(ds->shape_mu);
    ds->shapes[shape_key(g, which)] = Shape{shape->waves_per_group, shape->resident};
  } else {
    std::lock_guard<std::mutex> lk(ds->shape_mu);
    ds->shapes.erase(shape_key(g, which));
  }
  t_last_error.clear();
  return SF_OK;
}

int sf_get_launch_shape(const sf_desc *desc, int which, sf_launch_shape *out) {
  Geom g;
  int rc = make_geom(desc, &g);
  if (rc) return rc;
  if ((which != 0 && which != 1) || !out) return fail(SF_EINVAL, "which must be 0 or 1 and out non-NULL");
  DeviceState *ds;
  if ((rc = device_state(&ds))) return rc;
  Shape r;
  if ((rc = resolved_shape(*ds, g, which, stored_shape(*ds, g, which), &r))) return rc;
  out->waves_per_group = r.waves;
  out->resident = r.resident;
  t_last_error.clear();
  return SF_OK;
}

int sf_tune_image(const sf_desc *desc, const uint8_t *d_pixels, void *d_public, uint8_t *d_private,
                  const sf_exceptions *exc, int8_t *d_residual, const sf_aes_ctr *aes, uint8_t *d_restored,
                  uint32_t *d_status, void *stream, sf_launch_shape *best_frag, sf_launch_shape *best_defrag,
                  float *frag_ms, float *defrag_ms) {
  Geom g;
  int rc = make_geom(desc, &g);
  if (rc) return rc;
  if ((rc = check_call(g, d_pixels, d_public, d_private, exc, d_residual))) return rc;
  if (!d_restored || ((uintptr_t)d_restored & 7u)) return fail(SF_EINVAL, "d_restored must be an 8-byte aligned buffer");
  DeviceState *ds;
  if ((rc = device_state(&ds))) return rc;
  AesArgs a;
  make_aes_args(aes, &a);
  hipStream_t st = (hipStream_t)stream;
  auto run = [&](int which, const Shape &sh) {
    if (which == 0)
      return g.precision == SF_FP32
                 ? launch_frag_fp32(*ds, g, d_pixels, (float *)d_public, d_private, exc, a, d_status, sh, st)
                 : launch_frag_lp(*ds, g, d_pixels, d_public, d_private, exc, (uint8_t *)d_residual, a, d_status, sh,
                                  st);
    return g.precision == SF_FP32
               ? launch_defrag_fp32(*ds, g, (const float *)d_public, d_private, exc, a, d_restored, sh, st)
               : launch_defrag_lp(*ds, g, d_public, d_private, exc, (const uint8_t *)d_residual, a, d_restored,
                                  d_status, sh, st);
  };
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t he;
  if ((he = hipEventCreate(&e0)) != hipSuccess) return hip_fail(he, "hipEventCreate");
  if ((he = hipEventCreate(&e1)) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return hip_fail(he, "hipEventCreate");
  }
  static const uint32_t waves[] = {1, 2, 4, 6, 8};
  constexpr int kRounds = 2, kTimed = 5;
  Shape best[2] = {};
  float best_ms[2] = {0.0f, 0.0f};
  for (int which = 0; which < 2 && rc == SF_OK; ++which) {
    // defrag is timed on fragments made in frag's chosen shape
    if (which == 1 && (rc = run(0, best[0]))) break;
    Shape cand[10];
    float cand_ms[10];
    int nc = 0;
    for (uint32_t res = 0; res < 2; ++res)
      for (uint32_t w : waves) {
        Shape sh{w, res}, r;
        if (resolved_shape(*ds, g, which, sh, &r) == SF_OK) {  // shapes that do not fit are no candidates
          cand[nc] = sh;
          cand_ms[nc++] = 0.0f;
        }
      }
    if (!nc) {
      rc = fail(SF_ENOTSUP, "no launch shape fits this selection on this device");
      break;
    }
    for (int round = 0; round < kRounds && rc == SF_OK; ++round)
      for (int c = 0; c < nc && rc == SF_OK; ++c) {
        if ((rc = run(which, cand[c]))) break;
        if ((he = hipEventRecord(e0, st)) != hipSuccess) {
          rc = hip_fail(he, "hipEventRecord");
          break;
        }
        for (int i = 0; i < kTimed && rc == SF_OK; ++i) rc = run(which, cand[c]);
        if (rc) break;
        float ms = 0.0f;
        if ((he = hipEventRecord(e1, st)) != hipSuccess || (he = hipEventSynchronize(e1)) != hipSuccess ||
            (he = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) {
          rc = hip_fail(he, "timing a launch shape");
          break;
        }
        ms /= (float)kTimed;
        if (round == 0 || ms < cand_ms[c]) cand_ms[c] = ms;
      }
    if (rc) break;
    int b = 0;
    for (int c = 1; c < nc; ++c)
      if (cand_ms[c] < cand_ms[b]) b = c;
    best[which] = cand[b];
    best_ms[which] = cand_ms[b];
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  {
    std::lock_guard<std::mutex> lk(ds->shape_mu);
    ds->shapes[shape_key(g, 0)] = best[0];
    ds->shapes[shape_key(g, 1)] = best[1];
  }
  // leave the buffers holding a frag and a defrag in the chosen shapes
  if ((rc = run(0, best[0])) || (rc = run(1, best[1]))) return rc;
  if ((he = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(he, "hipStreamSynchronize");
  if (best_frag) *best_frag = sf_launch_shape{best[0].waves, best[0].resident};
  if (best_defrag) *best_defrag = sf_launch_shape{best[1].waves, best[1].resident};
  if (frag_ms) *frag_ms = best_ms[0];
  if (defrag_ms) *defrag_ms = best_ms[1];
  t_last_error.clear();
  return SF_OK;
}

size_t sf_batch_workspace_bytes(uint32_t n_items) { return batch_workspace_bytes(n_items); }

int sf_batch_plan(const sf_batch_item *items, uint32_t n_items, const uint8_t *key, void *d_workspace,
                  size_t workspace_bytes, void *stream) {
  if (!items || n_items == 0) return fail(SF_EINVAL, "empty batch");
  if (!d_workspace) return fail(SF_EINVAL, "NULL workspace");
  DeviceState *ds;
  int rc = device_state(&ds);
  if (rc) return rc;
  rc = batch_plan(*ds, items, n_items, key, d_workspace, workspace_bytes, (hipStream_t)stream);
  if (rc == SF_OK) t_last_error.clear();
  return rc;
}

static int batch_run_api(const void *d_workspace, int which, const sf_batch_tuning *tuning, uint32_t *d_status,
                         void *stream) {
  if (!d_workspace) return fail(SF_EINVAL, "NULL workspace");
  DeviceState *ds;
  int rc = device_state(&ds);
  if (rc) return rc;
  rc = batch_run(*ds, d_workspace, which, tuning, d_status, (hipStream_t)stream);
  if (rc == SF_OK) t_last_error.clear();
  return rc;
}

int sf_frag_batch(const void *d_workspace, const sf_batch_tuning *tuning, uint32_t *d_status, void *stream) {
  return batch_run_api(d_workspace, 0, tuning, d_status, stream);
}

int sf_defrag_batch(const void *d_workspace, const sf_batch_tuning *tuning, uint32_t *d_status, void *stream) {
  return batch_run_api(d_workspace, 1, tuning, d_status, stream);
}

int sf_batch_autotune(const void *d_workspace, sf_batch_tuning *best, float *best_ms, void *stream) {
  if (!d_workspace || !best) return fail(SF_EINVAL, "NULL argument");
  DeviceState *ds;
  int rc = device_state(&ds);
  if (rc) return rc;
  rc = batch_autotune(*ds, d_workspace, best, best_ms, (hipStream_t)stream);
  if (rc == SF_OK) t_last_error.clear();
  return rc;
}

// ---- wavelet variant
static int dwt_geom(uint32_t H, uint32_t W, uint32_t C, Geom *g) {
  if (H == 0 || W == 0 || H % 8 || W % 8) return fail(SF_ESHAPE, "height and width must be positive multiples of 8");
  if (C == 0) return fail(SF_ESHAPE, "channels must be >= 1");
  const uint64_t samples = (uint64_t)H * W * C;
  if (samples >= (1ull << 32)) return fail(SF_ESHAPE, "image must hold fewer than 2^32 samples");
  g->H = H;
  g->W = W;
  g->C = C;
  g->Bx = W / 8;
  g->By = H / 8;
  g->nb = samples / 64;
  g->ntiles = (uint32_t)((g->nb + 63) / 64);
  g->mask = 0;
  g->npriv = 4;
  g->npub = 60;
  g->precision = SF_FP32;
  return SF_OK;
}

int sf_dwt_fragment_sizes(uint32_t H, uint32_t W, uint32_t C, size_t *public_bytes, size_t *private_bytes) {
  Geom g;
  int rc = dwt_geom(H, W, C, &g);
  if (rc) return rc;
  if (public_bytes) *public_bytes = (size_t)g.nb * 60u * 2u;
  if (private_bytes) *private_bytes = (size_t)g.nb * 4u * 2u;
  return SF_OK;
}

int dwt_frag_image(uint32_t H, uint32_t W, uint32_t C, const uint8_t *d_pixels, int16_t *d_public,
                   uint8_t *d_private, const sf_aes_ctr *aes, void *stream) {
  Geom g;
  int rc = dwt_geom(H, W, C, &g);
  if (rc) return rc;
  if (!d_pixels || !d_public || !d_private) return fail(SF_EINVAL, "NULL buffer");
  if ((rc = check_alignment(d_pixels, d_public, d_private))) return rc;
  DeviceState *ds;
  if ((rc = device_state(&ds))) return rc;
  AesArgs a;
  make_aes_args(aes, &a);
  rc = launch_dwt_frag(*ds, g, d_pixels, d_public, d_private, a, (hipStream_t)stream);
  if (rc == SF_OK) t_last_error.clear();
  return rc;
}

int dwt_defrag_image(uint32_t H, uint32_t W, uint32_t C, const int16_t *d_public, const uint8_t *d_private,
                     const sf_aes_ctr *aes, uint8_t *d_pixels, void *stream) {
  Geom g;
  int rc = dwt_geom(H, W, C, &g);
  if (rc) return rc;
  if (!d_pixels || !d_public || !d_private) return fail(SF_EINVAL, "NULL buffer");
  if ((rc = check_alignment(d_pixels, d_public, d_private))) return rc;
  DeviceState *ds;
  if ((rc = device_state(&ds))) return rc;
  AesArgs a;
  make_aes_args(aes, &a);
  rc = launch_dwt_defrag(*ds, g, d_public, d_private, a, d_pixels, (hipStream_t)stream);
  if (rc == SF_OK) t_last_error.clear();
  return rc;
}

// ---- pixel-domain formats
static int pixel_geom(const sf_desc *desc, Geom *g) {
  int rc = make_geom(desc, g);
  if (rc) return rc;
  if (g->precision != SF_FP32) return fail(SF_EINVAL, "pixel-domain formats are integer only: precision must be SF_FP32");
  if (g->npriv > (uint32_t)kPixMaxPriv) return fail(SF_ERANGE, "pixel-domain formats take at most 16 private coefficients");
  return SF_OK;
}

static int pixel_flags(int flags) {
  if (flags & ~(SF_LEVEL_STRONG | SF_STORAGE_8BIT)) return fail(SF_EINVAL, "unknown pixel-format flags");
  return SF_OK;
}

int sf_pixel_fragment_sizes(const sf_desc *desc, int flags, size_t *public_bytes, size_t *private_bytes) {
  Geom g;
  int rc = pixel_geom(desc, &g);
  if (rc || (rc = pixel_flags(flags))) return rc;
  const PixLayout l = pixel_layout(g, flags);
  if (public_bytes) *public_bytes = (size_t)g.nb * 64u;
  if (private_bytes) *private_bytes = (size_t)(g.ntiles - 1u) * l.stride + l.last_bytes;
  return SF_OK;
}

int pixel_frag_image(const sf_desc *desc, int flags, const uint8_t *d_pixels, uint8_t *d_public, uint8_t *d_private,
                     const sf_aes_ctr *aes, void *stream) {
  Geom g;
  int rc = pixel_geom(desc, &g);
  if (rc || (rc = pixel_flags(flags))) return rc;
  if (!d_pixels || !d_public || !d_private) return fail(SF_EINVAL, "NULL buffer");
  if ((rc = check_alignment(d_pixels, d_public, d_private))) return rc;
  DeviceState *ds;
  if ((rc = device_state(&ds))) return rc;
  AesArgs a;
  make_aes_args(aes, &a);
  rc = launch_pixel_frag(*ds, g, flags, d_pixels, d_public, d_private, a, (hipStream_t)stream);
  if (rc == SF_OK) t_last_error.clear();
  return rc;
}

int pixel_defrag_image(const sf_desc *desc, int flags, const uint8_t *d_public, const uint8_t *d_private,
                       const sf_aes_ctr *aes, uint8_t *d_pixels, void *stream) {
  Geom g;
  int rc = pixel_geom(desc, &g);
  if (rc || (rc = pixel_flags(flags))) return rc;
  if (!d_pixels || !d_public || !d_private) return fail(SF_EINVAL, "NULL buffer");
  if ((rc = check_alignment(d_pixels, d_public, d_private))) return rc;
  DeviceState *ds;
  if ((rc = device_state(&ds))) return rc;
  AesArgs a;
  make_aes_args(aes, &a);
  rc = launch_pixel_defrag(*ds, g, flags, d_public, d_private, a, d_pixels, (hipStream_t)stream);
  if (rc == SF_OK) t_last_error.clear();
  return rc;
}

// ---- security statistics
size_t sf_stats_workspace_bytes(void) { return stats_workspace_bytes(); }

int sf_security_stats_compute(const uint8_t *d_x, const uint8_t *d_y, uint32_t H, uint32_t W, uint32_t C, void *d_ws,
                              size_t ws_bytes, sf_security_stats *d_out, float *d_block_entropy, void *stream) {
  if (!d_x || !d_y || !d_ws || !d_out) return fail(SF_EINVAL, "NULL buffer");
  if (H == 0 || W == 0 || H % 8 || W % 8) return fail(SF_ESHAPE, "height and width must be positive multiples of 8");
  if (C == 0) return fail(SF_ESHAPE, "channels must be >= 1");
  if ((uint64_t)H * W * C >= (1ull << 32)) return fail(SF_ESHAPE, "image must hold fewer than 2^32 samples");
  if (((uintptr_t)d_x | (uintptr_t)d_y | (uintptr_t)d_ws) & 15u) return fail(SF_EINVAL, "buffers must be 16-byte aligned");
  if (((uintptr_t)d_out & 7u) || ((uintptr_t)d_block_entropy & 3u)) return fail(SF_EINVAL, "misaligned output");
  if (ws_bytes < stats_workspace_bytes()) return fail(SF_EINVAL, "workspace too small");
  DeviceState *ds;
  int rc = device_state(&ds);
  if (rc) return rc;
  rc = launch_security_stats(*ds, d_x, d_y, H, W, C, d_ws, d_out, d_block_entropy, (hipStream_t)stream);
  if (rc == SF_OK) t_last_error.clear();
  return rc;
}

// ---- differentiation form
static int sm_ptrs(const void *a, const void *b) {
  if (!a || !b) return fail(SF_EINVAL, "NULL buffer");
  if (((uintptr_t)a | (uintptr_t)b) & 15u) return fail(SF_EINVAL, "buffers must be 16-byte aligned");
  return SF_OK;
}

size_t sf_softmask_workspace_bytes(uint32_t B, uint32_t H, uint32_t W) {
  DeviceState *ds;
  if (device_state(&ds)) return 0;
  return softmask_workspace_bytes(*ds, B, H, W);
}

int sf_softmask_forward(const float *d_x, uint32_t B, uint32_t H, uint32_t W, const float *d_logits,
                        float *d_public, double *d_stats, void *d_workspace, size_t workspace_bytes, void *stream) {
  int rc = sm_ptrs(d_x, d_stats);
  if (rc) return rc;
  if (!d_logits || !d_workspace || ((uintptr_t)d_public & 15u)) return fail(SF_EINVAL, "NULL or misaligned argument");
  DeviceState *ds;
  if ((rc = device_state(&ds))) return rc;
  rc = softmask_forward(*ds, d_x, B, H, W, d_logits, d_public, d_stats, d_workspace, workspace_bytes,
                        (hipStream_t)stream);
  if (rc == SF_OK) t_last_error.clear();
  return rc;
}

int sf_softmask_forward_noalloc(const float *d_x, uint32_t B, uint32_t H, uint32_t W, const float *d_logits,
                                float *d_public, double *d_stats, void *stream) {
  int rc = sm_ptrs(d_x, d_stats);
  if (rc) return rc;
  if (!d_logits || ((uintptr_t)d_public & 15u)) return fail(SF_EINVAL, "NULL or misaligned argument");
  DeviceState *ds;
  if ((rc = device_state(&ds))) return rc;
  rc = softmask_forward_noalloc(*ds, d_x, B, H, W, d_logits, d_public, d_stats, (hipStream_t)stream);
  if (rc == SF_OK) t_last_error.clear();
  return rc;
}

int sf_softmask_corr_stats(const float *d_x, const float *d_public, uint32_t B, uint32_t H, uint32_t W,
                           double *d_stats, void *d_workspace, size_t workspace_bytes, void *stream) {
  int rc = sm_ptrs(d_x, d_public);
  if (rc) return rc;
  if (!d_stats || !d_workspace) return fail(SF_EINVAL, "NULL argument");
  DeviceState *ds;
  if ((rc = device_state(&ds))) return rc;
  rc = softmask_corr_stats(*ds, d_x, d_public, B, H, W, d_stats, d_workspace, workspace_bytes, (hipStream_t)stream);
  if (rc == SF_OK) t_last_error.clear();
  return rc;
}

int sf_softmask_loss(const double *d_stats, int mode, const float *d_logits, uint32_t B, uint32_t H, uint32_t W,
                     float lam, float budget, double *d_loss, float *d_grad_logits, float *d_grad_budget,
                     float *d_gcoef, void *stream) {
  if (!d_stats || !d_logits || !d_loss) return fail(SF_EINVAL, "NULL argument");
  if (mode != 0 && mode != 1) return fail(SF_EINVAL, "mode must be 0 or 1");
  if (mode == 1 && d_grad_logits) return fail(SF_EINVAL, "closed-form gradient needs mode 0 statistics");
  DeviceState *ds;
  int rc = device_state(&ds);
  if (rc) return rc;
  rc = softmask_loss(d_stats, mode, d_logits, B, H, W, lam, budget, d_loss, d_grad_logits, d_grad_budget, d_gcoef,
                     (hipStream_t)stream);
  if (rc == SF_OK) t_last_error.clear();
  return rc;
}

int sf_softmask_corr_grad(const float *d_x, const float *d_public, uint32_t B, uint32_t H, uint32_t W,
                          const float *d_gcoef, const double *d_scale, float *d_grad_public, const float *d_grad_budget,
                          float *d_grad_logits, void *stream) {
  int rc = sm_ptrs(d_x, d_public);
  if (rc) return rc;
  if (!d_gcoef || !d_grad_public || ((uintptr_t)d_grad_public & 15u)) return fail(SF_EINVAL, "NULL or misaligned");
  if (!d_grad_budget != !d_grad_logits) return fail(SF_EINVAL, "budget gradient input and output go together");
  DeviceState *ds;
  if ((rc = device_state(&ds))) return rc;
  rc = softmask_corr_grad(d_x, d_public, B, H, W, d_gcoef, d_scale, d_grad_public, d_grad_budget, d_grad_logits,
                          (hipStream_t)stream);
  if (rc == SF_OK) t_last_error.clear();
  return rc;
}

int sf_softmask_tune(const double *d_stats, uint32_t B, uint32_t H, uint32_t W, float lam, float budget,
                     uint32_t steps, float lr, float *d_logits, double *d_loss_trace, uint64_t *d_private_mask,
                     uint32_t n_private, void *stream) {
  if (!d_stats || !d_logits) return fail(SF_EINVAL, "NULL argument");
  DeviceState *ds;
  int rc = device_state(&ds);
  if (rc) return rc;
  rc = softmask_tune(d_stats, B, H, W, lam, budget, steps, lr, d_logits, d_loss_trace, d_private_mask, n_private,
                     (hipStream_t)stream);
  if (rc == SF_OK) t_last_error.clear();
  return rc;
}

int sf_softmask_backward(const float *d_x, const float *d_grad_public, uint32_t B, uint32_t H, uint32_t W,
                         const float *d_logits, float *d_grad_logits, void *d_workspace, size_t workspace_bytes,
                         void *stream) {
  int rc = sm_ptrs(d_x, d_grad_public);
  if (rc) return rc;
  if (!d_logits || !d_grad_logits || !d_workspace) return fail(SF_EINVAL, "NULL argument");
  DeviceState *ds;
  if ((rc = device_state(&ds))) return rc;
  rc = softmask_backward(*ds, d_x, d_grad_public, B, H, W, d_logits, d_grad_logits, d_workspace, workspace_bytes,
                         (hipStream_t)stream);
  if (rc == SF_OK) t_last_error.clear();
  return rc;
}

int encrypt_private(const sf_aes_ctr *aes, uint64_t first_block, const uint8_t *d_in, uint8_t *d_out,
                    size_t nbytes, void *stream) {
  if (!aes) return fail(SF_EINVAL, "aes is NULL");
  if (nbytes == 0) return SF_OK;
  if (!d_in || !d_out) return fail(SF_EINVAL, "NULL buffer");
  if (nbytes > (1ull << 40)) return fail(SF_ERANGE, "nbytes too large");
  DeviceState *ds;
  int rc = device_state(&ds);
  if (rc) return rc;
  AesArgs a;
  make_aes_args(aes, &a);
  rc = launch_ctr(*ds, a, first_block, d_in, d_out, nbytes, (hipStream_t)stream);
  if (rc == SF_OK) t_last_error.clear();
  return rc;
}

}  // extern "C"
