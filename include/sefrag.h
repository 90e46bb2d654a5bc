/*
 * sefrag.h -- C ABI of the MI355X (gfx950) selective-fragmentation library.
 *
 * Method: the "first level of protection" of the report "Data Protection:
 * Combining Fragmentation, Encryption, and Dispersion" (Memmi, Kapusta,
 * Lambein, Qiu), Sec. 6.3.1 and Fig. 6: every 8x8 block of an 8-bit image is
 * transformed with the orthonormal DCT-II (Sec. 6.1, 6.4.2); a selected set of
 * low-frequency coefficients (by default DC and the first five zigzag AC
 * coefficients [0,0],[0,1],[1,0],[2,0],[1,1],[0,2]; the ratio is user-tunable,
 * Sec. 6.2.1/6.3.1) is stored as integers (Sec. 6.4.3 "11-bit storage", held in
 * int16) and encrypted with AES-128 (here in counter mode); the remaining
 * coefficients form the public fragment.  Defragmentation (Sec. 5.2, Fig. 3)
 * decrypts, merges, inverse-transforms and restores every sample exactly.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Pointers named d_* are DEVICE pointers, allocated and owned by the caller;
 *   all other pointers are host pointers read during the call only.
 * - Alignment: pixel buffers 8 bytes, fragment and residual buffers 16 bytes
 *   (torch and hipMalloc allocations satisfy both); otherwise SF_EINVAL.
 * - Work is enqueued asynchronously on `stream` (a hipStream_t; NULL is the
 *   default stream).  Host-side validation is synchronous: a negative return
 *   code means nothing was enqueued.
 * - The library allocates no memory per call.  On first use of a device it
 *   uploads small constant tables (AES T-tables, integer DCT basis) and keeps
 *   them until the process ends; its code object also holds, per device, the
 *   1 MiB static scratch array of sf_softmask_forward_noalloc.
 * - Errors: SF_* codes below; sf_last_error() returns a thread-local message
 *   for the last failing call on this thread.
 * - Device-detected conditions are OR-ed into *d_status (one uint32 the caller
 *   zeroes when it wants a fresh reading and reads after synchronising).
 *
 * Image and fragment layouts
 * --------------------------
 * Image: uint8 planar [channels][height][width], row-major; height and width
 * are positive multiples of 8 (otherwise SF_ESHAPE); channels >= 1; the
 * total sample count must stay below 2^32.  Blocks are numbered
 * b = (c*By + by)*Bx + bx with By = height/8, Bx = width/8.
 *
 * Coefficient selection: bit z of private_mask marks zigzag position z (JPEG
 * order over [u=row frequency, v=column frequency]) as private.  DC plus the
 * first k AC coefficients is private_mask = (1 << (k+1)) - 1.
 *
 * Fragments use the 64-block tile-interleaved layout: tile t covers blocks
 * 64t .. 64t+n_t-1 with n_t = min(64, nb - 64t); value j (0 <= j < P) of block
 * 64t+i is element 64*t*P + j*n_t + i.  Values within a block are in zigzag
 * order (private: the P = popcount(mask) private positions; public: the other
 * 64 - P positions).
 *   public fragment : float32 (SF_FP32) or fp16 / bf16 (SF_FP16 / SF_BF16)
 *                     DCT coefficients.  SF_FP16 / SF_BF16 split each tile
 *                     into halves of m_0 = min(32, n_t) and m_1 = n_t - m_0
 *                     blocks: public value j of block 64t + 32h + i (i <
 *                     m_h) is element 64*t*P + h*P*m_0 + j*m_h + i, so each
 *                     half's values are one contiguous run.
 *   private fragment: int16 little-endian integers q = round_half_even(
 *                     sum_p x_p * round_half_even(2^20 B[n][p]) / 2^20 ),
 *                     as one byte stream, AES-128-CTR encrypted with counter
 *                     blocks ctr0 + i (128-bit big-endian increment, NIST
 *                     SP 800-38A) when an sf_aes_ctr is given.
 */
#ifndef SEFRAG_H
#define SEFRAG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ---- */
#define SF_OK 0
#define SF_EINVAL (-1)    /* null pointer, unknown enum, empty private mask          */
#define SF_ESHAPE (-2)    /* height/width not positive multiples of 8, or too large  */
#define SF_ERANGE (-3)    /* a size or capacity argument out of range                */
#define SF_EHIP (-5)      /* HIP runtime error; see sf_last_error()                  */
#define SF_ENOTSUP (-6)   /* no gfx950 device, or an unsupported combination         */

/* ---- bits OR-ed into *d_status by the kernels ---- */
#define SF_STATUS_EXC_OVERFLOW 0x1u  /* more exceptions than capacity; *d_count holds the number found */
#define SF_STATUS_RESIDUAL_RANGE 0x2u /* reserved (no longer raised: residuals beyond +-1 go to the exception slots) */
#define SF_STATUS_PRIVATE_RANGE 0x4u  /* a private integer fell outside int16 (never for uint8 input)  */

/* ---- precisions of the transform and of the public fragment ---- */
#define SF_FP32 0u  /* plain form: FP32 vector DCT, sparse exception list                 */
#define SF_FP16 1u  /* reduced precision: fp16 MFMA DCT, 2-bit residual codes + exceptions */
#define SF_BF16 2u  /* reduced precision: bf16 MFMA DCT (hi/lo basis), as SF_FP16          */

typedef struct sf_desc {
  uint32_t height;        /* rows per channel, multiple of 8                         */
  uint32_t width;         /* columns, multiple of 8                                  */
  uint32_t channels;      /* planar channels (1 = gray, 3 = RGB)                     */
  uint32_t precision;     /* SF_FP32, SF_FP16 or SF_BF16                             */
  uint64_t private_mask;  /* bit z set: zigzag position z is private; must be nonzero */
} sf_desc;

/* AES-128 key and the 16-byte initial counter block (host memory, copied by
 * value during the call).  The key schedule is expanded on the host. */
typedef struct sf_aes_ctr {
  uint8_t key[16];
  uint8_t ctr0[16];
} sf_aes_ctr;

/* Exceptions: in the plain (SF_FP32) form, samples whose reconstruction
 * from the stored fragments would not round back to the input (the report
 * notes the DCT cannot guarantee losslessness, Sec. 6.4.3/6.8); in the
 * reduced-precision forms, samples whose residual is not -1, 0 or +1 (their
 * residual code is 2).  They are kept in per-tile slots of one device buffer
 * of sf_exception_bytes() bytes:
 *   uint16 count[ntiles]                        (ntiles = ceil(blocks / 64))
 *   uint16 pos[ntiles][per_tile]   = block-in-tile * 64 + 8*y + x
 *   uint8  value[ntiles][per_tile] = the sample's value
 * each part starting on a 16-byte boundary.  frag_image writes every count
 * (a count above per_tile means slots were lost: SF_STATUS_EXC_OVERFLOW);
 * defrag_image reads them.  No clearing is needed between calls.
 * In the plain form, selections of DC plus at most 4 AC coefficients never
 * produce exceptions; for them the buffer is neither read nor written and
 * may be NULL.  The reduced-precision forms always need the buffer (on
 * natural and synthetic images their slots stay empty). */
typedef struct sf_exceptions {
  void *d_buf;        /* device buffer, sf_exception_bytes(desc, per_tile) bytes  */
  uint32_t per_tile;  /* slots per 64-block tile, 1 .. 4096                      */
} sf_exceptions;

/* Library version string. */
const char *sf_version(void);
/* Message for a return code. */
const char *sf_strerror(int code);
/* Thread-local description of the last failure on this thread ("" if none). */
const char *sf_last_error(void);

/* Byte sizes of the fragments for a descriptor (host only, no GPU needed).
 * Any output pointer may be NULL.  residual_bytes is 0 for SF_FP32 and
 * channels*height*width/4 (2 bits per sample) for the reduced-precision
 * forms.
 * Returns SF_OK, SF_EINVAL or SF_ESHAPE. */
int sf_fragment_sizes(const sf_desc *desc, size_t *public_bytes, size_t *private_bytes, size_t *residual_bytes);

/* Byte size of an exception buffer with per_tile slots per tile (host only).
 * *needed is set to 0 when the selection can never produce exceptions
 * (plain form only).
 * Returns SF_OK, SF_EINVAL, SF_ESHAPE or SF_ERANGE (per_tile > 4096). */
int sf_exception_bytes(const sf_desc *desc, uint32_t per_tile, size_t *bytes, int *needed);

/* Initialise the library on the current HIP device (optional; every entry
 * point does it lazily).  Returns SF_OK, SF_ENOTSUP or SF_EHIP. */
int sf_init(void);

/* frag_image -- fragmentation (Sec. 6.3.1, Fig. 6: DCT 8x8, selection,
 * AES on the private part, public part left plain; Sec. 6.5.2: all steps on
 * the GPU).
 *   d_pixels  : input image, C*H*W bytes.
 *   d_public  : out, public fragment (size from sf_fragment_sizes).
 *   d_private : out, private fragment, encrypted when aes != NULL.
 *   exc       : exception slots; required (non-NULL, with a buffer) unless
 *               sf_exception_bytes reports them not needed.
 *   d_residual: SF_FP16/SF_BF16 only: out, the residual codes of
 *               r = x - clamp(round(y)), y the inverse transform of the
 *               stored fragments: 2 bits per sample, code 0 (r = 0),
 *               1 (r = +1), 3 (r = -1), 2 (|r| >= 2: the sample is in the
 *               exception slots).  One 16-byte record per block (block b at
 *               byte 16 b); sample (y, x) of the block at bit
 *               32 (2 (x / 4) + y / 4) + 8 (x % 4) + 2 (y % 4).  NULL for
 *               SF_FP32.
 *   aes       : key + initial counter, or NULL to leave the private integers
 *               in clear.
 *   d_status  : device word for SF_STATUS_* bits (may be NULL).
 * Output buffers must not overlap the input. */
int frag_image(const sf_desc *desc, const uint8_t *d_pixels, void *d_public, uint8_t *d_private,
               const sf_exceptions *exc, int8_t *d_residual, const sf_aes_ctr *aes, uint32_t *d_status,
               void *stream);

/* defrag_image -- defragmentation (Sec. 5.2, Fig. 3): decrypt the private
 * fragment, merge with the public coefficients in zigzag order, inverse DCT,
 * round half to even, clamp to [0,255], then add the residual codes
 * (SF_FP16/SF_BF16) and put back the samples in the exception slots.
 * Restores the input
 * of the matching frag_image call bit for bit.  Arguments mirror frag_image;
 * d_pixels is the output. */
int defrag_image(const sf_desc *desc, const void *d_public, const uint8_t *d_private, const sf_exceptions *exc,
                 const int8_t *d_residual, const sf_aes_ctr *aes, uint8_t *d_pixels, uint32_t *d_status,
                 void *stream);

/* encrypt_private -- AES-128 in counter mode over an arbitrary device buffer
 * (Sec. 6.2.2/6.5.2: AES on the selected part; SP 800-38A counter mode):
 *   out[j] = in[j] XOR E_K(ctr0 + first_block + j/16)[j mod 16].
 * Encryption and decryption are the same call; d_in == d_out is allowed. */
int encrypt_private(const sf_aes_ctr *aes, uint64_t first_block, const uint8_t *d_in, uint8_t *d_out,
                    size_t nbytes, void *stream);

/* ---------------------------------------------------------------------
 * Launch shapes of frag_image / defrag_image and their tuner.  The same
 * data-parallel pass over 64-block tiles (Sec. 6.4.2: the DCT stage on the
 * GPU; Sec. 6.5.1: a series of images processed one after another) can be
 * launched in several shapes that give identical results; which is fastest
 * depends on the image size, the selection and the precision.  The library
 * keeps, per device, the shape to use for each (precision, private_mask,
 * size class) -- size class = ceil(log2(number of 64-block tiles)) -- and
 * falls back to the form's measured default where it has none.
 * ------------------------------------------------------------------- */

/* One launch shape.  Host struct. */
typedef struct sf_launch_shape {
  uint32_t waves_per_group; /* wavefronts per workgroup: 1, 2, 4, 6 or 8;
                               0 = the form's default (plain: 4 for frag,
                               and for defrag of 8 or more private
                               coefficients, else 2; reduced precision: the
                               largest that lets two workgroups share a
                               compute unit's LDS)                          */
  uint32_t resident;        /* 1: one resident generation of workgroups
                               (as many as the device holds at once) loops
                               over the tiles (the default of the reduced
                               precision, and of the plain form's defrag for
                               8 or more private coefficients); 0: the grid
                               gives each wavefront one tile (plain) or one
                               pair of tiles (reduced precision)            */
} sf_launch_shape;

/* sf_set_launch_shape -- the shape frag_image (which = 0) or defrag_image
 * (which = 1) uses on the current device for images of desc's precision,
 * private_mask and size class; shape = NULL forgets it (back to the
 * default).  Host only, synchronous.  SF_EINVAL for which not in {0, 1} or
 * waves_per_group not in {0, 1, 2, 4, 6, 8} or resident not in {0, 1};
 * SF_ENOTSUP when that many wavefronts' LDS does not fit one workgroup on
 * this device for desc's selection. */
int sf_set_launch_shape(const sf_desc *desc, int which, const sf_launch_shape *shape);

/* sf_get_launch_shape -- the shape that the next frag_image (which = 0) or
 * defrag_image (which = 1) for desc would use on the current device (the
 * stored one, else the default, resolved: waves_per_group is never 0).
 * Host only.  Returns SF_OK, SF_EINVAL / SF_ESHAPE for bad arguments, or
 * SF_ENOTSUP when no workgroup of this form fits the selection's LDS. */
int sf_get_launch_shape(const sf_desc *desc, int which, sf_launch_shape *out);

/* sf_tune_image -- times frag_image and then defrag_image of the image in
 * every shape that fits (waves_per_group 1, 2, 4, 6, 8 x resident 0, 1) on
 * `stream`: two rounds over the shapes, each shape one untimed and five
 * timed launches per round, a shape's time the lower of its two round
 * averages; stores the fastest of each direction as with
 * sf_set_launch_shape.  Arguments as in
 * frag_image (d_pixels in; d_public, d_private, exc, d_residual out) plus
 * d_restored, the output of defrag_image (must not overlap the others).
 * Synchronous: returns when the timing is done; on return the fragments and
 * d_restored hold a frag_image and a defrag_image in the chosen shapes.
 * best_frag / best_defrag (may be NULL) receive the shapes; frag_ms /
 * defrag_ms (may be NULL) their average times per launch.  The call
 * allocates a few HIP events. */
int sf_tune_image(const sf_desc *desc, const uint8_t *d_pixels, void *d_public, uint8_t *d_private,
                  const sf_exceptions *exc, int8_t *d_residual, const sf_aes_ctr *aes, uint8_t *d_restored,
                  uint32_t *d_status, void *stream, sf_launch_shape *best_frag, sf_launch_shape *best_defrag,
                  float *frag_ms, float *defrag_ms);

/* ---------------------------------------------------------------------
 * Batched form: many images of uneven sizes and selections (plain FP32
 * form) in one persistent kernel per direction.  Images are independent
 * pieces of data (the report's arbitrary data chunked into matrices and
 * processed block by block, Sec. 6.9.3; a series of images, Sec. 6.5.1),
 * each with its own counter block (a different IV per input, Sec. 6.10.6).
 * ------------------------------------------------------------------- */

/* One image of a batch.  Host struct; the pointers are device pointers
 * owned by the caller, with the layouts and alignments of frag_image. */
typedef struct sf_batch_item {
  uint32_t height, width, channels; /* as in sf_desc (multiples of 8)             */
  uint32_t exc_per_tile;            /* exception slots per tile (see sf_exceptions) */
  uint64_t private_mask;            /* as in sf_desc                                */
  const uint8_t *d_pixels;          /* frag input image (NULL: plan not for frag)   */
  uint8_t *d_restored;              /* defrag output image (NULL: not for defrag)   */
  float *d_public;                  /* FP32 public fragment                         */
  uint8_t *d_private;               /* private fragment                             */
  void *d_exc;                      /* exception buffer, or NULL if not needed      */
  uint8_t ctr0[16];                 /* this image's initial counter block           */
} sf_batch_item;

/* Launch shape of a batch run (workgroups of 4 wavefronts, one persistent
 * grid) over the batch's 64-block tiles, numbered image after image.
 * schedule 0, work queue: the run first clears a counter, then each
 * wavefront grabs tiles_per_grab consecutive tiles per atomic add.
 * schedule 1, static chunks: the tiles are cut into chunks of
 * 4 * tiles_per_grab consecutive tiles dealt round-robin to the workgroups,
 * the wavefronts of a workgroup taking every 4th tile of its chunk (faster on
 * large line-aligned images).  tiles_per_grab 0 = the schedule's default (8
 * queue, 2 static; at most 1024); workgroups_per_cu 0 = as many as fit.
 * reserved must be 0.  NULL tuning = {8, 0, 0, 0}.  Every shape gives the
 * same fragments. */
typedef struct sf_batch_tuning {
  uint32_t tiles_per_grab;
  uint32_t workgroups_per_cu;
  uint32_t schedule;
  uint32_t reserved;
} sf_batch_tuning;

/* Device workspace bytes for a plan of n_items images. */
size_t sf_batch_workspace_bytes(uint32_t n_items);

/* Validates the items and writes their descriptors, each image's first
 * global tile, a table from tile ranges to the images they fall in, and the
 * AES key (key = 16 host bytes, or NULL to leave private integers in clear)
 * into d_workspace (one copy from the host).  Synchronises `stream`
 * before returning (the host item array may be released afterwards).  Not
 * capturable into a graph; the run calls below are.  Returns SF_OK,
 * SF_EINVAL (bad item, with its index in sf_last_error), SF_ESHAPE,
 * SF_ERANGE (workspace too small) or SF_EHIP. */
int sf_batch_plan(const sf_batch_item *items, uint32_t n_items, const uint8_t *key, void *d_workspace,
                  size_t workspace_bytes, void *stream);

/* Fragment / defragment every image of the planned batch: one persistent
 * kernel on `stream` (the work-queue schedule adds a reset of its counter
 * before it).  Returns SF_EINVAL, launching nothing, for an unknown
 * schedule, a nonzero reserved field, or a plan with an item without the
 * direction's image buffer (d_pixels for frag, d_restored for defrag), and
 * SF_ERANGE for tiles_per_grab above 1024. */
int sf_frag_batch(const void *d_workspace, const sf_batch_tuning *tuning, uint32_t *d_status, void *stream);
int sf_defrag_batch(const void *d_workspace, const sf_batch_tuning *tuning, uint32_t *d_status, void *stream);

/* Autotuner: times frag + defrag of the planned batch for the work queue
 * with tiles_per_grab in {4,8,16,32} and the static schedule with {1,2,4,8},
 * each with workgroups_per_cu in {1,2,3} (one warm pass, two timed round
 * trips each) and returns the fastest; *best_ms = its round-trip time.
 * Runs the batch many times (outputs are rewritten with identical values).
 * Needs both d_pixels and d_restored on every item (else SF_EINVAL, nothing
 * launched). */
int sf_batch_autotune(const void *d_workspace, sf_batch_tuning *best, float *best_ms, void *stream);

/* ---------------------------------------------------------------------
 * Wavelet variant (Sec. 6.8-6.9, Eqs. (1)-(2), Fig. 18): every 8x8 block of
 * a planar uint8 image (samples read as x - 128, Sec. 6.9.4) goes through two
 * levels of the LeGall 5/3 integer lifting (rows, then columns; the second
 * level on the 4x4 low-low quarter; whole-sample symmetric extension).  The
 * 2x2 second-level low-low corner is the private fragment (Sec. 6.9.3: 4 of
 * 64 coefficients), int16 little endian, encrypted with AES-128-CTR as one
 * byte stream (as frag_image; aes may be NULL for plaintext); the other 60
 * coefficients, in row-major order of their positions, are the public
 * fragment, int16.  Both fragments use the tile-interleaved layout of
 * frag_image with P = 4 (private) and P = 60 (public) values per block.
 * Integer lifting is exactly invertible: defragmentation restores every
 * sample with no exception list or residual.  Buffers: pixels 8-byte
 * aligned, fragments 16-byte aligned, device memory owned by the caller;
 * errors as for frag_image.  Any byte data can be processed by viewing it as
 * a gray image of width W (Sec. 6.9.3, data-agnostic chunking).
 * ------------------------------------------------------------------- */

/* Host only: public and private fragment bytes of an H x W x C image. */
int sf_dwt_fragment_sizes(uint32_t height, uint32_t width, uint32_t channels, size_t *public_bytes,
                          size_t *private_bytes);

int dwt_frag_image(uint32_t height, uint32_t width, uint32_t channels, const uint8_t *d_pixels, int16_t *d_public,
                   uint8_t *d_private, const sf_aes_ctr *aes, void *stream);

int dwt_defrag_image(uint32_t height, uint32_t width, uint32_t channels, const int16_t *d_public,
                     const uint8_t *d_private, const sf_aes_ctr *aes, uint8_t *d_pixels, void *stream);

/* ---------------------------------------------------------------------
 * Pixel-domain formats of the report (Sec. 6.3.1-6.3.2, Sec. 6.4.3,
 * Figs. 6-8, Table 5).  desc as for frag_image with precision SF_FP32 (the
 * path is integer only) and at most 16 private coefficients (SF_ERANGE).
 *   private fragment: the private integers of frag_image (rule Q2, zigzag
 *     order), each in one field: DC unsigned in 11 bits (0..2040); AC a sign
 *     bit above a 10-bit magnitude (11-bit storage, |AC| <= 1020, exact) or,
 *     with SF_STORAGE_8BIT, above a 7-bit magnitude clamped to 127 (the
 *     report's lossy 8-bit storage, Sec. 6.4.3, Table 5).  A block's fields
 *     follow each other in a record of B bits (B = 11 P for 11-bit storage);
 *     the records of a 64-block tile form one little-endian bit stream
 *     (block i of the tile at bit B i); tile t starts at byte t * S,
 *     S = 16 ceil(8 B / 16) (zero padding up to the AES-block boundary); the
 *     last tile holds ceil(B n_t / 8) bytes.  The whole byte string is
 *     AES-128-CTR encrypted as in frag_image (aes NULL: plaintext).  The
 *     fields take 12.9 % of the image for P = 6 at 11 bits, 9.96 % at 8.
 *   public fragment: one byte per sample, same layout as the image:
 *     P(p) = (x(p) - R(p)) mod 256 with R(p) = floor((sum_j q_j
 *     rhe(2^16 B[n_j][p]) + 2^15) / 2^16), the integer inverse of the
 *     private part (rhe: round half to even).
 *     It stands for the inverse DCT of the remaining coefficients (private
 *     ones zeroed), which the report stores as bytes, and makes the round trip
 *     exact: x(p) = (R(p) + P(p)) mod 256.  P is always made from the exact
 *     integers; with 8-bit storage defrag uses the stored (clamped) ones, so
 *     blocks with a clamped AC come back as (x + R(stored) - R(exact)) mod 256.
 *   flags SF_LEVEL_STRONG (Sec. 6.3.2, Fig. 8): the 64 public bytes of each
 *     block are XORed with the SHA-512 digest (FIPS 180-4) of the block's
 *     stored private integers as int16 little endian, digest byte 8y + x on
 *     sample (y, x) of the block.  SF_LEVEL_FIRST (0) leaves them as they are.
 *     Flags combine with OR; frag and defrag must be given the same flags.
 * Buffers: device memory owned by the caller; pixels 8-byte aligned, public
 * and private 16-byte aligned (SF_EINVAL otherwise).  Kernels run on
 * stream; errors as for frag_image.
 * ------------------------------------------------------------------- */
#define SF_LEVEL_FIRST 0
#define SF_LEVEL_STRONG 1
#define SF_STORAGE_8BIT 2

/* Host only: public (C*H*W) and private fragment bytes for these flags. */
int sf_pixel_fragment_sizes(const sf_desc *desc, int flags, size_t *public_bytes, size_t *private_bytes);

int pixel_frag_image(const sf_desc *desc, int flags, const uint8_t *d_pixels, uint8_t *d_public,
                     uint8_t *d_private, const sf_aes_ctr *aes, void *stream);

int pixel_defrag_image(const sf_desc *desc, int flags, const uint8_t *d_public, const uint8_t *d_private,
                       const sf_aes_ctr *aes, uint8_t *d_pixels, void *stream);

/* ---------------------------------------------------------------------
 * Security statistics (Sec. 6.6, Sec. 6.10, Eqs. (3)-(4), Table 14) of a
 * protected byte image Y against its original X, both planar C x H x W
 * (H, W positive multiples of 8; fewer than 2^32 samples), e.g. X the input
 * and Y the public fragment of pixel_frag_image.  Written by the device into
 * *d_out (device memory; copy it to the host after the stream has run):
 *   hist_x, hist_y : byte histograms; chi2_y: sum (h - N/256)^2 / (N/256).
 *   entropy_x/_y, joint_entropy : Eq. (3) in bits over the samples and the
 *     pairs (x, y); mutual_information = H(X) + H(Y) - H(X,Y);
 *     nmi = mutual_information / sqrt(H(X) H(Y)).
 *   pair_x/_y[d] : exact moments (n, Sx, Sy, Sxx, Syy, Sxy) over every
 *     adjacent pair of a plane, d = horizontal, vertical, diagonal (x the
 *     upper / left sample), pooled over planes; corr_x/_y[d] their Pearson r
 *     (the report samples 10,000 or 4,096 pairs; this is the population).
 *   cross : (N, Sx, Sy, Sxx, Syy, Sxy) of X against Y; corr2 its Pearson r.
 *   bits_differing, dif = 100 bits_differing / (8 N) (also the key
 *     sensitivity measure of Sec. 6.10.6 when X, Y are two ciphertexts);
 *     psnr = 10 log10(255^2 N / sum (x - y)^2) (inf when X = Y).
 *   block_entropy_x/_y : mean, standard deviation, min, max over the 8x8
 *     blocks of Eq. (3) over the block's 64 samples (h = 8, at most 6).
 * d_block_entropy (optional, NULL to skip): 2 * C * (H/8) * (W/8) floats,
 * the block entropies of X then of Y, block order of frag_image.
 * d_ws: caller-owned device workspace of sf_stats_workspace_bytes() bytes,
 * 16-byte aligned; its first 65536 uint32 hold the joint histogram
 * (bin 256 x + y) after the call.  X and Y 16-byte aligned.  Errors:
 * SF_EINVAL (NULL, misaligned, workspace too small), SF_ESHAPE, SF_EHIP.
 * ------------------------------------------------------------------- */
typedef struct sf_security_stats {
  uint64_t samples;
  uint64_t hist_x[256];
  uint64_t hist_y[256];
  uint64_t pair_x[3][6];
  uint64_t pair_y[3][6];
  uint64_t cross[6];
  uint64_t bits_differing;
  double chi2_y;
  double entropy_x, entropy_y, joint_entropy, mutual_information, nmi;
  double corr_x[3], corr_y[3];
  double corr2, dif, psnr;
  double block_entropy_x[4], block_entropy_y[4];
} sf_security_stats;

size_t sf_stats_workspace_bytes(void);

int sf_security_stats_compute(const uint8_t *d_x, const uint8_t *d_y, uint32_t height, uint32_t width,
                              uint32_t channels, void *d_ws, size_t ws_bytes, sf_security_stats *d_out,
                              float *d_block_entropy, void *stream);

/* ---------------------------------------------------------------------
 * Differentiation form: a soft per-frequency selection mask
 * m_n = sigmoid(l_n) over the 64 natural frequencies n = 8u + v, and the
 * public image it leaves, P = IDCT(DCT(x) * (1 - m)) per 8x8 block (the
 * hard-mask case is the zero-padded public image of Sec. 6.3.1 / Fig. 7b).
 * Images: B planes of H x W float32 (H, W multiples of 8), contiguous.
 * The tuning objective is the mean over images of the squared Pearson
 * correlation of P and x (Sec. 6.6.2, population moments) plus
 * lam * (sum_n m_n - budget)^2.  Statistics are FP64.
 * ------------------------------------------------------------------- */

/* Device workspace bytes for the soft-mask calls on B x H x W images. */
size_t sf_softmask_workspace_bytes(uint32_t B, uint32_t H, uint32_t W);

/* Forward: d_public (may be NULL) <- P; d_stats (B x 65 doubles) <- per image
 * E_n = sum over blocks of DCT(x)_n^2 (n = 0..63), then sum x. */
int sf_softmask_forward(const float *d_x, uint32_t B, uint32_t H, uint32_t W, const float *d_logits,
                        float *d_public, double *d_stats, void *d_workspace, size_t workspace_bytes, void *stream);

/* Allocation-free variant of sf_softmask_forward, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight tuning loops,
 * harnesses that forbid allocation): the same kernels and results, with the
 * per-workgroup partial sums in a static device array of 1 MiB that the
 * library holds on each device it runs on until the process ends.  No
 * workspace argument; no hipMalloc/hipFree or allocating library call.
 * Returns SF_ERANGE, launching nothing, when the batch needs more partial
 * sums than the array holds (sf_softmask_workspace_bytes(B, H, W) > 1 MiB,
 * about B > 2000 images); otherwise as sf_softmask_forward.  Calls on one
 * device share its array: calls that overlap on one device (different
 * streams, or different host threads) race and must be serialised by the
 * caller; calls in one stream are ordered and safe. */
int sf_softmask_forward_noalloc(const float *d_x, uint32_t B, uint32_t H, uint32_t W, const float *d_logits,
                                float *d_public, double *d_stats, void *stream);

/* Correlation statistics of an arbitrary P: d_stats (B x 5 doubles) <-
 * sum x, sum P, sum xP, sum x^2, sum P^2 per image. */
int sf_softmask_corr_stats(const float *d_x, const float *d_public, uint32_t B, uint32_t H, uint32_t W,
                           double *d_stats, void *d_workspace, size_t workspace_bytes, void *stream);

/* Loss from statistics.  mode 0: d_stats from sf_softmask_forward (P implied
 * by the mask, correlation terms by Parseval: sum xP = sum_n (1-m_n) E_n,
 * sum P^2 = sum_n (1-m_n)^2 E_n, mean P = (1-m_0) mean x); mode 1: d_stats
 * from sf_softmask_corr_stats.  Outputs (each may be NULL): *d_loss;
 * d_grad_logits (64, mode 0 only): the whole dL/dl in closed form;
 * d_grad_budget (64): the budget term's dL/dl; d_gcoef (B x 4 floats:
 * a, b, mean x, mean P) with dL/dP = a (x - mean x) + b (P - mean P). */
int sf_softmask_loss(const double *d_stats, int mode, const float *d_logits, uint32_t B, uint32_t H, uint32_t W,
                     float lam, float budget, double *d_loss, float *d_grad_logits, float *d_grad_budget,
                     float *d_gcoef, void *stream);

/* d_grad_public <- s * (a (x - mean x) + b (P - mean P)) per image, from the
 * d_gcoef written by sf_softmask_loss, with s = *d_scale (a device double,
 * the upstream gradient of the loss; NULL means 1).  If d_grad_budget (64
 * floats from sf_softmask_loss) is given, d_grad_logits (64) <- s times it. */
int sf_softmask_corr_grad(const float *d_x, const float *d_public, uint32_t B, uint32_t H, uint32_t W,
                          const float *d_gcoef, const double *d_scale, float *d_grad_public, const float *d_grad_budget,
                          float *d_grad_logits, void *stream);

/* The tuning loop on the statistics of sf_softmask_forward (the mode 0
 * closed form needs no further pass over the images): `steps` Adam updates
 * (beta1 0.9, beta2 0.999, eps 1e-8, step size lr) of d_logits in place, the
 * loss before each update into d_loss_trace (steps doubles, may be NULL),
 * then the n_private largest logits (ties to the lower n) hardened into a
 * private_mask for frag_image at *d_private_mask (may be NULL): logit n
 * belongs to natural frequency n, and bit z is set for the zigzag position z
 * of each chosen frequency.  Minimising the correlation of the public image
 * with the input under the budget picks the coefficients whose removal hides
 * the most (Sec. 6.6.2 measures protection by this correlation). */
int sf_softmask_tune(const double *d_stats, uint32_t B, uint32_t H, uint32_t W, float lam, float budget,
                     uint32_t steps, float lr, float *d_logits, double *d_loss_trace, uint64_t *d_private_mask,
                     uint32_t n_private, void *stream);

/* Adjoint (backward) of the forward for an arbitrary upstream gradient
 * G = dL/dP: d_grad_logits (64) <- sigmoid'(l_n) * (- sum over images and
 * blocks of DCT(G)_n DCT(x)_n), the transposed transform applied to G. */
int sf_softmask_backward(const float *d_x, const float *d_grad_public, uint32_t B, uint32_t H, uint32_t W,
                         const float *d_logits, float *d_grad_logits, void *d_workspace, size_t workspace_bytes,
                         void *stream);

#ifdef __cplusplus
}
#endif
#endif /* SEFRAG_H */
