// Internal host-side declarations of the library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <mutex>
#include <string>
#include <tuple>

#include "sefrag.h"
#include "sf_device.h"

namespace sf {

// MFMA operand tables: f16 forward, f16 inverse, bf16 forward hi/lo, bf16
// inverse; each 2 M-tiles x 4 K-steps x 64 lanes x 4 words.
constexpr int kLpTables = 5;
constexpr int kLpTableWords = 2 * 4 * 64 * 4;
void build_lp_tables(const double *basis, uint32_t (*lp)[kLpTableWords]);

// Host-generated constant tables (tables.cpp), independent of any device.
struct HostTables {
  uint32_t aes_t0[256];                  // T0[x] = (2S, S, S, 3S) bytes, little-endian word
  uint8_t sbox[256];                     // FIPS-197 S-box
  uint32_t q2[64 * kQ2RowWords];         // integer basis limbs, see q2_acc()
  int32_t q2_int[64 * 64];               // round_half_even(2^20 B[n][p])
  int32_t inv16[64 * 64];               // round_half_even(2^16 B[n][p]), pixel-domain inverse
  float cert_m[64];                      // max_p |B[n][p]| (rounded up), per natural index
  float cert_e[64];                      // 255 * sum_p |Bq/2^20 - B| (rounded up)
  DctK dct;                              // butterfly constants
  double basis[64 * 64];                 // B[n][p] (long double rounded to double)
  // MFMA operand tables of the reduced-precision form, per-lane order (lp.hip)
  uint32_t lp[kLpTables][kLpTableWords];
};
const HostTables &host_tables();
void aes_expand_key(const uint8_t key[16], uint32_t rk[44]);
// Certificate threshold and whether a selection can ever need the
// reconstruction check (false for DC + up to 4 AC).
float cert_threshold();
bool mask_needs_check(uint64_t mask);

// Launch shape of the single-image kernels (resolved: waves >= 1).
struct Shape {
  uint32_t waves;     // wavefronts per workgroup
  uint32_t resident;  // 1: one resident generation of workgroups loops over the tiles
};
// (precision, private mask, size class, direction)
using ShapeKey = std::tuple<uint32_t, uint64_t, uint32_t, int>;

// Per-device state: device copies of the tables.
struct DeviceState {
  int device = -1;
  int num_cu = 0;
  uint32_t *d_aes_t0 = nullptr;
  uint32_t *d_q2 = nullptr;
  uint32_t *d_lp = nullptr;  // kLpTables x kLpTableWords
  size_t max_lds_per_block = 65536;
  void *d_sm_scratch = nullptr;  // this device's copy of the soft-mask scratch array
  std::mutex shape_mu;           // guards shapes
  std::map<ShapeKey, Shape> shapes;  // tuned or set launch shapes
};
// Lazily initialise the current device; returns SF_OK or an error code.
int device_state(DeviceState **out);

// Error reporting (thread-local message).
int fail(int code, const std::string &msg);
int hip_fail(hipError_t e, const char *what);

// Validated geometry of one image.
struct Geom {
  uint32_t H, W, C, Bx, By;
  uint64_t nb;       // number of 8x8 blocks
  uint32_t ntiles;   // ceil(nb / 64)
  uint64_t mask;
  uint32_t npriv, npub;
  uint32_t precision;
};
int make_geom(const sf_desc *desc, Geom *g);

// AES parameters as passed to kernels.
struct AesArgs {
  AesKey key;
  uint64_t ctr_hi, ctr_lo;
  uint32_t enabled;
};
void make_aes_args(const sf_aes_ctr *aes, AesArgs *a);

// Byte layout of an exception buffer: uint16 count per tile, then
// per_tile uint16 positions and per_tile uint8 values per tile, each part
// padded to 16 bytes.
struct ExcLayout {
  size_t pos_offset, val_offset, total;
};
ExcLayout exc_layout(const Geom &g, uint32_t per_tile);
constexpr uint32_t kMaxExcPerTile = 4096;

// Launch shapes (api.hip): the stored shape of (g, which = 0 frag / 1
// defrag), else the form's default (waves = 0: chosen by the launcher).
Shape stored_shape(DeviceState &ds, const Geom &g, int which);
// Workgroup LDS (static + dynamic) of a shape, for the fit check (plain.hip,
// lp.hip).
size_t plain_lds_bytes(const Geom &g, int which, uint32_t waves);
size_t lp_lds_bytes(const Geom &g, int which, uint32_t waves);
// Default wavefronts per workgroup of the reduced-precision kernels.
uint32_t lp_default_waves(const DeviceState &ds, const Geom &g, int which);
// Default shape of the plain kernels: 4 waves per workgroup, resident, for
// selections of 8 or more private coefficients; 2 waves, one tile per wave,
// for the lighter ones (measured on the 4096^2 RGB DC + 5 AC and the 8192^2
// DC + 9 AC workloads).
inline bool plain_heavy(const Geom &g) { return g.npriv >= 8; }
// Default waves per workgroup of the plain kernels: frag 4 (one tile each,
// up to 5 resident per SIMD by registers and LDS), defrag 4 from 8 private
// coefficients on, else 2.
inline uint32_t plain_default_waves(const Geom &g, int which) { return which == 0 || plain_heavy(g) ? 4u : 2u; }

// Launchers (plain.hip, aes.hip).
int launch_frag_fp32(const DeviceState &ds, const Geom &g, const uint8_t *pix, float *pub, uint8_t *priv,
                     const sf_exceptions *exc, const AesArgs &aes, uint32_t *status, const Shape &sh,
                     hipStream_t stream);
int launch_defrag_fp32(const DeviceState &ds, const Geom &g, const float *pub, const uint8_t *priv,
                       const sf_exceptions *exc, const AesArgs &aes, uint8_t *pix, const Shape &sh,
                       hipStream_t stream);
// Reduced-precision (MFMA fp16 / bf16 + 2-bit residual codes and exception
// slots) form (lp.hip).
int launch_frag_lp(const DeviceState &ds, const Geom &g, const uint8_t *pix, void *pub, uint8_t *priv,
                   const sf_exceptions *exc, uint8_t *residual, const AesArgs &aes, uint32_t *status,
                   const Shape &sh, hipStream_t stream);
int launch_defrag_lp(const DeviceState &ds, const Geom &g, const void *pub, const uint8_t *priv,
                     const sf_exceptions *exc, const uint8_t *residual, const AesArgs &aes, uint8_t *pix,
                     uint32_t *status, const Shape &sh, hipStream_t stream);
// Batched form (batch.hip).
size_t batch_workspace_bytes(uint32_t n);
int batch_plan(const DeviceState &ds, const sf_batch_item *items, uint32_t n, const uint8_t *key, void *d_ws,
               size_t ws_bytes, hipStream_t stream);
int batch_run(const DeviceState &ds, const void *d_ws, int which, const sf_batch_tuning *tuning, uint32_t *status,
              hipStream_t stream);
int batch_autotune(const DeviceState &ds, const void *d_ws, sf_batch_tuning *best, float *best_ms,
                   hipStream_t stream);
// Wavelet variant (dwt.hip).
int launch_dwt_frag(const DeviceState &ds, const Geom &g, const uint8_t *pix, int16_t *pub, uint8_t *priv,
                    const AesArgs &aes, hipStream_t stream);
int launch_dwt_defrag(const DeviceState &ds, const Geom &g, const int16_t *pub, const uint8_t *priv,
                      const AesArgs &aes, uint8_t *pix, hipStream_t stream);

// Pixel-domain formats: 11-bit private fields, byte public part, optional
// SHA-512 strong level (pixel.hip).  At most kPixMaxPriv private coefficients.
constexpr int kPixMaxPriv = 16;
struct PixLayout {
  uint32_t ac_bits;     // 10 (11-bit fields) or 7 (8-bit fields)
  uint32_t rec_bits;    // bits per block
  uint32_t stride;      // bytes per full tile (multiple of 16)
  uint32_t last_bytes;  // bytes of the last tile
};
PixLayout pixel_layout(const Geom &g, int flags);
int launch_pixel_frag(const DeviceState &ds, const Geom &g, int flags, const uint8_t *pix, uint8_t *pub,
                      uint8_t *priv, const AesArgs &aes, hipStream_t stream);
int launch_pixel_defrag(const DeviceState &ds, const Geom &g, int flags, const uint8_t *pub, const uint8_t *priv,
                        const AesArgs &aes, uint8_t *pix, hipStream_t stream);

// Security statistics (stats.hip).
size_t stats_workspace_bytes();
int launch_security_stats(const DeviceState &ds, const uint8_t *x, const uint8_t *y, uint32_t H, uint32_t W,
                          uint32_t C, void *ws, sf_security_stats *out, float *block_entropy, hipStream_t stream);

// Differentiation form (softmask.hip).
size_t softmask_workspace_bytes(const DeviceState &ds, uint32_t B, uint32_t H, uint32_t W);
// Allocation-free forward: partial sums in a static device array of
// kSoftmaskScratchBytes (softmask_scratch_address gives the current device's
// copy; called once per device at initialisation).
constexpr size_t kSoftmaskScratchBytes = size_t(1) << 20;
int softmask_scratch_address(void **ptr);
int softmask_forward_noalloc(const DeviceState &ds, const float *x, uint32_t B, uint32_t H, uint32_t W,
                             const float *logits, float *p_out, double *stats, hipStream_t stream);
int softmask_forward(const DeviceState &ds, const float *x, uint32_t B, uint32_t H, uint32_t W, const float *logits,
                     float *p_out, double *stats, void *ws, size_t ws_bytes, hipStream_t stream);
int softmask_corr_stats(const DeviceState &ds, const float *x, const float *p, uint32_t B, uint32_t H, uint32_t W,
                        double *stats, void *ws, size_t ws_bytes, hipStream_t stream);
int softmask_backward(const DeviceState &ds, const float *x, const float *gpub, uint32_t B, uint32_t H, uint32_t W,
                      const float *logits, float *grad_logits, void *ws, size_t ws_bytes, hipStream_t stream);
int softmask_loss(const double *stats, int mode, const float *logits, uint32_t B, uint32_t H, uint32_t W, float lam,
                  float budget, double *loss, float *grad_logits, float *grad_budget, float *gcoef,
                  hipStream_t stream);
int softmask_corr_grad(const float *x, const float *p, uint32_t B, uint32_t H, uint32_t W, const float *gcoef,
                       const double *scale, float *g, const float *grad_budget, float *grad_out, hipStream_t stream);
int softmask_tune(const double *stats, uint32_t B, uint32_t H, uint32_t W, float lam, float budget, uint32_t steps,
                  float lr, float *logits, double *trace, uint64_t *mask, uint32_t n_private, hipStream_t stream);
int launch_ctr(const DeviceState &ds, const AesArgs &aes, uint64_t first_block, const uint8_t *in, uint8_t *out,
               size_t nbytes, hipStream_t stream);

}  // namespace sf
