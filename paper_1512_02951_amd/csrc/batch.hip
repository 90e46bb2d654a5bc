// Batched form: many images of uneven sizes and selections in one persistent
// kernel per direction.
//
//   plan (host, once):  validate the items, write per-image descriptors,
//                       the images' first global tiles, a bucket table that
//                       narrows a tile's image to a few candidates, and the
//                       AES key into the caller's device workspace.
//   run  (graph-safe):  one persistent grid per direction runs the same
//                       per-tile body as the single-image kernels
//                       (plain_tile.h) on every global tile, with the
//                       geometry, selection, fragments and counter block of
//                       the tile's image.  Two schedules:
//                       work queue (default): a kernel clears a counter,
//                       then each wave grabs tiles_per_grab consecutive
//                       tiles per atomic.
//                       static chunks: the global tiles are cut
//                       into chunks of 4 * tiles_per_grab consecutive tiles,
//                       dealt round-robin to the workgroups, the 4 waves of
//                       a workgroup taking interleaved tiles of its chunk.
//                       The tiles in flight form one dense window, as in the
//                       single-image kernels.  Faster on large line-aligned
//                       images (the queue's waves work through their grabs
//                       one tile after another, so the tiles in flight are
//                       spread out), slower on the batching workload's many
//                       unaligned ones.
//
// The tuner times candidate (schedule, tiles_per_grab, workgroups per CU)
// triples on the planned batch and reports the fastest.
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "plain_tile.h"

namespace sf {
namespace {

constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;

struct BatchDesc {
  TileGeom g;
  uint8_t *out;
  float *pub;
  uint8_t *priv;
  ExcSlots exc;
  uint64_t ctr_hi, ctr_lo;
};

// Device workspace layout (all offsets multiples of 16 bytes).
struct BatchHeader {
  uint32_t n;            // images
  uint32_t enc;          // AES enabled
  uint32_t total_tiles;  // filled by the scan
  uint32_t max_npriv;
  uint32_t queue[4];     // work counters of the queue schedule (frag, defrag)
  uint32_t bucket_shift; // tile t lies in image buckets[t >> bucket_shift] ..
  uint32_t nbuckets;     //   buckets[(t >> bucket_shift) + 1]
  uint32_t pad[2];
  AesKey key;
};

__host__ __device__ inline size_t align16(size_t v) { return (v + 15u) & ~(size_t)15u; }

// Bucket table entries (+1): 16 per image rounded up to a power of two, at
// least 1024 and at most 2^22, so that a bucket holds a few images at most
// unless the images' tile counts are very uneven.
__host__ __device__ inline uint32_t bucket_count(uint32_t n) {
  uint64_t want = 16ull * n, nb = 1024;
  while (nb < want && nb < (1ull << 22)) nb <<= 1;
  return (uint32_t)nb;
}

struct WsLayout {
  size_t desc, offsets, buckets, total;
};
__host__ __device__ inline WsLayout ws_layout(uint32_t n) {
  WsLayout L;
  L.desc = align16(sizeof(BatchHeader));
  L.offsets = L.desc + align16(sizeof(BatchDesc) * (size_t)n);
  L.buckets = L.offsets + align16(4u * ((size_t)n + 1u));
  L.total = L.buckets + align16(4u * ((size_t)bucket_count(n) + 1u));
  return L;
}

__global__ void batch_reset_kernel(uint8_t *ws, int which) { reinterpret_cast<BatchHeader *>(ws)->queue[which] = 0u; }

// Descriptor words through the scalar cache (the table is read-only while a
// batch kernel runs), so the image's geometry and pointers sit in SGPRs.
__device__ __forceinline__ BatchDesc load_desc(const BatchDesc *p) {
  static_assert(sizeof(BatchDesc) % 4 == 0, "descriptor must be whole words");
  constexpr int kWords = (int)(sizeof(BatchDesc) / 4);
  uint32_t w[kWords];
  const cu32_ptr src = as_const(reinterpret_cast<const uint32_t *>(p));
#pragma unroll
  for (int i = 0; i < kWords; ++i) w[i] = src[i];
  BatchDesc d;
  __builtin_memcpy(&d, w, sizeof(d));
  return d;
}

// Image holding global tile gt: the last i with offsets[i] <= gt, searched
// between the bounds that gt's bucket gives.
__device__ __forceinline__ uint32_t find_image(const uint32_t *offs, const uint32_t *bk, uint32_t shift,
                                               uint32_t gt) {
  const uint32_t b = gt >> shift;
  uint32_t lo = bk[b], hi = bk[b + 1] + 1u;  // offs[lo] <= gt < offs[hi]
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (offs[mid] <= gt) lo = mid;
    else hi = mid;
  }
  return lo;
}

constexpr int kSchedQueue = 0, kSchedStatic = 1;
constexpr uint32_t kDefaultChunkTiles = 2;

// Runs body(tile, desc) for every tile of the batch, in the schedule kSched
// (see the top of this file).
template <int kSched, class Body>
__device__ __forceinline__ void batch_loop(uint8_t *ws, uint32_t n, int which, uint32_t tiles_per_grab, int lane,
                                           Body &&body) {
  const WsLayout L = ws_layout(n);
  BatchHeader *hd = reinterpret_cast<BatchHeader *>(ws);
  const BatchDesc *descs = reinterpret_cast<const BatchDesc *>(ws + L.desc);
  const uint32_t *offs = reinterpret_cast<const uint32_t *>(ws + L.offsets);
  const uint32_t *bk = reinterpret_cast<const uint32_t *>(ws + L.buckets);
  const uint32_t total = hd->total_tiles, shift = hd->bucket_shift;
  if (kSched == kSchedStatic) {
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t G = gridDim.x, chunk = kWaves * tiles_per_grab;
    const uint32_t nchunks = (uint32_t)(((uint64_t)total + chunk - 1) / chunk);
    for (uint32_t c = blockIdx.x; c < nchunks; c += G) {
      const uint32_t base = c * chunk, end = base + min(chunk, total - base);
      uint32_t img = __builtin_amdgcn_readfirstlane(find_image(offs, bk, shift, base));
      for (uint32_t gt = base + wave; gt < end; gt += kWaves) {
        while (offs[img + 1] <= gt) ++img;
        img = __builtin_amdgcn_readfirstlane(img);
        body(gt - offs[img], load_desc(descs + img));
      }
    }
  } else {
    for (;;) {
      uint32_t w = 0;
      if (lane == 0) w = atomicAdd(&hd->queue[which], tiles_per_grab);
      w = __builtin_amdgcn_readfirstlane(__shfl(w, 0, 64));
      if (w >= total) break;
      const uint32_t end = min(w + tiles_per_grab, total);
      uint32_t img = __builtin_amdgcn_readfirstlane(find_image(offs, bk, shift, w));
      for (uint32_t gt = w; gt < end; ++gt) {
        while (offs[img + 1] <= gt) ++img;
        img = __builtin_amdgcn_readfirstlane(img);
        body(gt - offs[img], load_desc(descs + img));
      }
    }
  }
}

struct BatchArgs {
  uint8_t *ws;
  uint32_t n;
  uint32_t tiles_per_grab;
  uint32_t lds_priv_bytes;
  uint32_t *status;
  const uint32_t *aes_t0;
  const uint32_t *q2;
  float cert_thr;
  DctK K;
};

// Selections with a compiled body; kAny adds the run-time body for any other
// mask (the plan picks the kernels without it when no image needs it: that
// body's registers would otherwise size every tile's).
__host__ __device__ constexpr bool compiled_mask(uint64_t mask) {
  return mask == (1ull << 2) - 1 || mask == (1ull << 3) - 1 || mask == (1ull << 6) - 1 || mask == (1ull << 10) - 1;
}

template <bool kAny, class F>
__device__ __forceinline__ void dispatch_mask(uint64_t mask, F &&f) {
  switch (mask) {
    case (1ull << 2) - 1: f(MaskPrefix<2>{}); break;
    case (1ull << 3) - 1: f(MaskPrefix<3>{}); break;
    case (1ull << 6) - 1: f(MaskPrefix<6>{}); break;
    case (1ull << 10) - 1: f(MaskPrefix<10>{}); break;
    default:
      if constexpr (kAny) f(MaskRuntime{});
      break;
  }
}

// Per-wave LDS of the batched frag: private bytes, the quantiser stage, and
// the quantiser's B operand for the mask of the image in hand (recomputed
// when the wave moves to an image with another mask).
constexpr uint32_t kBatchQ2Bytes = kQ2StageBytes + 64u * sizeof(Q2Operands);

template <int kSched, bool kAny>
__global__ __launch_bounds__(kThreads, 3) void frag_batch_kernel(BatchArgs a) {
  __shared__ AesLds s_aes;
  extern __shared__ __attribute__((aligned(16))) uint8_t s_dyn[];
  const int lane = threadIdx.x & 63;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const BatchHeader *hd = reinterpret_cast<const BatchHeader *>(a.ws);
  const uint32_t enc = hd->enc;
  if (enc) aes_load_tables(s_aes, a.aes_t0, hd->key, threadIdx.x, kThreads);
  __syncthreads();
  uint8_t *lp = s_dyn + wave * (a.lds_priv_bytes + kBatchQ2Bytes);
  uint8_t *stage = lp + a.lds_priv_bytes;
  Q2Operands *wq = reinterpret_cast<Q2Operands *>(stage + kQ2StageBytes);
  uint64_t qmask = 0;  // mask whose operands wq holds (masks are never 0)
  // the body must be inlined: its buffer resources and table pointers live in
  // scalar registers, which an outlined call could not guarantee
  batch_loop<kSched>(a.ws, a.n, 0, a.tiles_per_grab, lane, [&](uint32_t t, const BatchDesc &d) __attribute__((always_inline)) {
    FragOut o;
    o.pub = d.pub;
    o.priv = d.priv;
    o.exc = d.exc;
    o.status = a.status;
    o.q2 = a.q2;
    o.cert_thr = a.cert_thr;
    const TileLane L = tile_lane(d.g, t, lane);
    uint32_t xs[16];
    load_block(d.g, L, xs);
    // the compiled selections have at most 9 private AC coefficients
    const bool mfma_q2 = !kAny || __builtin_popcountll(d.g.mask & ~1ull) <= kQ2MfmaMaxAc;
    dispatch_mask<kAny>(d.g.mask, [&](auto mp) __attribute__((always_inline)) {
      using MP = decltype(mp);
      if (mfma_q2) {
        if (d.g.mask != qmask) {
          wave_lds_sync();
          wq[lane] = q2_operands(a.q2, private_ac<MP>(d.g.mask, lane & 15), lane);
          wave_lds_sync();
          qmask = d.g.mask;
        }
        frag_tile<MP, true>(d.g, o, t, L, xs, lane, lp, s_aes, enc, d.ctr_hi, d.ctr_lo, a.K, stage, &wq[lane]);
      } else {
        frag_tile<MP, false>(d.g, o, t, L, xs, lane, lp, s_aes, enc, d.ctr_hi, d.ctr_lo, a.K);
      }
    });
  });
}

template <int kSched, bool kAny>
__global__ __launch_bounds__(kThreads, 3) void defrag_batch_kernel(BatchArgs a) {
  __shared__ AesLds s_aes;
  extern __shared__ __attribute__((aligned(16))) uint8_t s_dyn[];
  const int lane = threadIdx.x & 63;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const BatchHeader *hd = reinterpret_cast<const BatchHeader *>(a.ws);
  const uint32_t enc = hd->enc;
  if (enc) aes_load_tables(s_aes, a.aes_t0, hd->key, threadIdx.x, kThreads);
  __syncthreads();
  uint8_t *lp = s_dyn + wave * a.lds_priv_bytes;
  batch_loop<kSched>(a.ws, a.n, 1, a.tiles_per_grab, lane, [&](uint32_t t, const BatchDesc &d) __attribute__((always_inline)) {
    DefragIn in;
    in.pix_out = d.out;
    in.pub = d.pub;
    in.priv = d.priv;
    in.exc = d.exc;
    const TileLane L = tile_lane(d.g, t, lane);
    dispatch_mask<kAny>(d.g.mask, [&](auto mp) __attribute__((always_inline)) {
      defrag_tile<decltype(mp)>(d.g, in, t, L, lane, lp, s_aes, enc, d.ctr_hi, d.ctr_lo, a.K);
    });
  });
}

// Host copy of the plan's facts needed at launch time (kept per workspace).
struct PlanInfo {
  const void *ws = nullptr;
  uint32_t n = 0, max_npriv = 0;
  uint64_t total_tiles = 0;
  bool all_pixels = true;    // every item has d_pixels: frag can run
  bool all_restored = true;  // every item has d_restored: defrag can run
  bool any_mask = false;     // some item's selection has no compiled body
};
std::vector<PlanInfo> g_plans;  // guarded by g_plan_mu
std::mutex g_plan_mu;

int find_plan(const void *ws, PlanInfo *out) {
  std::lock_guard<std::mutex> lk(g_plan_mu);
  for (const PlanInfo &p : g_plans)
    if (p.ws == ws) {
      *out = p;
      return SF_OK;
    }
  return fail(SF_EINVAL, "workspace has no batch plan (call sf_batch_plan first)");
}

int launch_batch(const DeviceState &ds, const PlanInfo &p, int which, const sf_batch_tuning *tuning,
                 uint32_t *status, hipStream_t stream) {
  BatchArgs a;
  a.ws = (uint8_t *)p.ws;
  a.n = p.n;
  const uint32_t sched = tuning ? tuning->schedule : (uint32_t)kSchedQueue;
  if ((sched != (uint32_t)kSchedStatic && sched != (uint32_t)kSchedQueue) || (tuning && tuning->reserved))
    return fail(SF_EINVAL, "schedule must be 0 (work queue) or 1 (static chunks), reserved 0");
  // defaults: what the tuner picks on the batching workload
  a.tiles_per_grab = tuning && tuning->tiles_per_grab ? tuning->tiles_per_grab
                                                      : (sched == (uint32_t)kSchedStatic ? kDefaultChunkTiles : 8u);
  a.lds_priv_bytes = (2u * p.max_npriv * 64u + 15u) & ~15u;
  a.status = status;
  a.aes_t0 = ds.d_aes_t0;
  a.q2 = ds.d_q2;
  a.cert_thr = cert_threshold();
  a.K = host_tables().dct;
  if (a.tiles_per_grab > 1024) return fail(SF_ERANGE, "tiles_per_grab must be at most 1024");
  const size_t lds = (size_t)kWaves * (a.lds_priv_bytes + (which == 0 ? kBatchQ2Bytes : 0u));
  // kernels by [direction][schedule][any mask]
  using Kern = void (*)(BatchArgs);
  static const Kern kerns[2][2][2] = {
      {{frag_batch_kernel<kSchedQueue, false>, frag_batch_kernel<kSchedQueue, true>},
       {frag_batch_kernel<kSchedStatic, false>, frag_batch_kernel<kSchedStatic, true>}},
      {{defrag_batch_kernel<kSchedQueue, false>, defrag_batch_kernel<kSchedQueue, true>},
       {defrag_batch_kernel<kSchedStatic, false>, defrag_batch_kernel<kSchedStatic, true>}}};
  const bool st = sched == (uint32_t)kSchedStatic;
  const Kern kern = kerns[which][st ? 1 : 0][p.any_mask ? 1 : 0];
  const void *fn = (const void *)kern;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kThreads, lds) != hipSuccess || per_cu < 1) per_cu = 1;
  if (tuning && tuning->workgroups_per_cu) per_cu = tuning->workgroups_per_cu < (uint32_t)per_cu ? (int)tuning->workgroups_per_cu : per_cu;
  uint64_t need = (p.total_tiles + (uint64_t)kWaves * a.tiles_per_grab - 1) / ((uint64_t)kWaves * a.tiles_per_grab);
  uint64_t grid = (uint64_t)ds.num_cu * (uint64_t)per_cu;
  if (need < grid) grid = need;
  if (grid < 1) grid = 1;
  if (!st) hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(1), 0, stream, a.ws, which);
  hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(kThreads), lds, stream, a);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SF_OK : hip_fail(e, "batch kernel launch");
}

}  // namespace

size_t batch_workspace_bytes(uint32_t n) { return ws_layout(n).total; }

int batch_plan(const DeviceState &ds, const sf_batch_item *items, uint32_t n, const uint8_t *key, void *d_ws,
               size_t ws_bytes, hipStream_t stream) {
  const WsLayout L = ws_layout(n);
  if (ws_bytes < L.total) return fail(SF_ERANGE, "batch workspace too small (see sf_batch_workspace_bytes)");
  if ((uintptr_t)d_ws & 15u) return fail(SF_EINVAL, "workspace must be 16-byte aligned");
  std::vector<uint8_t> host(L.total, 0);
  BatchHeader *hd = reinterpret_cast<BatchHeader *>(host.data());
  BatchDesc *descs = reinterpret_cast<BatchDesc *>(host.data() + L.desc);
  uint32_t *offs = reinterpret_cast<uint32_t *>(host.data() + L.offsets);
  uint32_t *bk = reinterpret_cast<uint32_t *>(host.data() + L.buckets);
  hd->n = n;
  hd->enc = key ? 1u : 0u;
  if (key) aes_expand_key(key, hd->key.rk);
  uint64_t total = 0;
  uint32_t max_npriv = 1;
  bool all_pixels = true, all_restored = true, any_mask = false;
  for (uint32_t i = 0; i < n; ++i) {
    const sf_batch_item &it = items[i];
    sf_desc d;
    d.height = it.height;
    d.width = it.width;
    d.channels = it.channels;
    d.precision = SF_FP32;
    d.private_mask = it.private_mask;
    Geom g;
    if (int rc = make_geom(&d, &g)) return fail(rc, "item " + std::to_string(i) + ": " + ::sf_last_error());
    if (!it.d_pixels && !it.d_restored) return fail(SF_EINVAL, "item " + std::to_string(i) + ": no image buffer");
    all_pixels = all_pixels && it.d_pixels;
    all_restored = all_restored && it.d_restored;
    if (!it.d_private || (g.npub && !it.d_public))
      return fail(SF_EINVAL, "item " + std::to_string(i) + ": NULL fragment pointer");
    if (((uintptr_t)it.d_pixels | (uintptr_t)it.d_restored) & 7u || ((uintptr_t)it.d_public | (uintptr_t)it.d_private) & 15u)
      return fail(SF_EINVAL, "item " + std::to_string(i) + ": misaligned buffer");
    BatchDesc &bd = descs[i];
    bd.g = tile_geom(g, it.d_pixels);
    bd.out = it.d_restored;
    bd.pub = it.d_public;
    bd.priv = it.d_private;
    sf_exceptions ex{it.d_exc, it.exc_per_tile};
    bd.exc = ExcSlots{};
    bd.exc.check = mask_needs_check(g.mask) ? 1u : 0u;
    if (bd.exc.check) {
      if (!it.d_exc || it.exc_per_tile == 0 || it.exc_per_tile > kMaxExcPerTile || ((uintptr_t)it.d_exc & 15u))
        return fail(SF_EINVAL, "item " + std::to_string(i) + ": this selection needs an exception buffer");
      bd.exc = exc_slots(g, &ex);
    }
    uint64_t hi = 0, lo = 0;
    for (int b = 0; b < 8; ++b) hi = (hi << 8) | it.ctr0[b];
    for (int b = 8; b < 16; ++b) lo = (lo << 8) | it.ctr0[b];
    bd.ctr_hi = hi;
    bd.ctr_lo = lo;
    any_mask = any_mask || !compiled_mask(g.mask);
    offs[i] = (uint32_t)total;
    total += g.ntiles;
    if (total >= (1ull << 31)) return fail(SF_ERANGE, "batch holds too many tiles");
    if (g.npriv > max_npriv) max_npriv = g.npriv;
  }
  offs[n] = (uint32_t)total;
  hd->total_tiles = (uint32_t)total;
  hd->max_npriv = max_npriv;
  // bucket b covers tiles [b << shift, (b + 1) << shift); bk[b] is the image
  // of its first tile (of the last tile for buckets past the end), so a
  // tile of bucket b lies in one of the images bk[b] .. bk[b + 1]
  const uint32_t nb = bucket_count(n);
  uint32_t shift = 0;
  while (((total - 1) >> shift) >= nb) ++shift;
  hd->bucket_shift = shift;
  hd->nbuckets = nb;
  for (uint32_t b = 0, img = 0; b <= nb; ++b) {
    const uint64_t t = std::min<uint64_t>((uint64_t)b << shift, total - 1);
    while (offs[img + 1] <= t) ++img;
    bk[b] = img;
  }
  hipError_t e = hipMemcpyAsync(d_ws, host.data(), L.total, hipMemcpyHostToDevice, stream);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(batch plan)");
  if ((e = hipStreamSynchronize(stream)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize(batch plan)");
  PlanInfo p;
  p.ws = d_ws;
  p.n = n;
  p.max_npriv = max_npriv;
  p.total_tiles = total;
  p.all_pixels = all_pixels;
  p.all_restored = all_restored;
  p.any_mask = any_mask;
  std::lock_guard<std::mutex> lk(g_plan_mu);
  for (PlanInfo &q : g_plans)
    if (q.ws == d_ws) {
      q = p;
      return SF_OK;
    }
  g_plans.push_back(p);
  (void)ds;
  return SF_OK;
}

int batch_run(const DeviceState &ds, const void *d_ws, int which, const sf_batch_tuning *tuning, uint32_t *status,
              hipStream_t stream) {
  PlanInfo p;
  if (int rc = find_plan(d_ws, &p)) return rc;
  if (which == 0 && !p.all_pixels) return fail(SF_EINVAL, "batch frag needs d_pixels on every item of the plan");
  if (which == 1 && !p.all_restored) return fail(SF_EINVAL, "batch defrag needs d_restored on every item of the plan");
  return launch_batch(ds, p, which, tuning, status, stream);
}

int batch_autotune(const DeviceState &ds, const void *d_ws, sf_batch_tuning *best, float *best_ms,
                   hipStream_t stream) {
  PlanInfo p;
  if (int rc = find_plan(d_ws, &p)) return rc;
  if (!p.all_pixels || !p.all_restored)
    return fail(SF_EINVAL, "batch autotune runs both directions: every item needs d_pixels and d_restored");
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return fail(SF_EHIP, "hipEventCreate failed");
  // tiles per grab (queue; single-tile grabs wait on the one counter's
  // atomics) or per wave and chunk (static)
  static const uint32_t grabs[2][4] = {{4, 8, 16, 32}, {1, 2, 4, 8}};
  float best_t = 1e30f;
  sf_batch_tuning best_c{8, 0, (uint32_t)kSchedQueue, 0};
  int rc = SF_OK;
  for (uint32_t sched = 0; sched < 2 && rc == SF_OK; ++sched)
  for (uint32_t wpc = 1; wpc <= 3 && rc == SF_OK; ++wpc)
    for (uint32_t gi = 0; gi < 4 && rc == SF_OK; ++gi) {
      sf_batch_tuning c{grabs[sched][gi], wpc, sched, 0};
      // one untimed pass, then two timed round trips
      for (int w = 0; w < 1 && rc == SF_OK; ++w) {
        rc = launch_batch(ds, p, 0, &c, nullptr, stream);
        if (rc == SF_OK) rc = launch_batch(ds, p, 1, &c, nullptr, stream);
      }
      (void)hipEventRecord(e0, stream);
      for (int r = 0; r < 2 && rc == SF_OK; ++r) {
        rc = launch_batch(ds, p, 0, &c, nullptr, stream);
        if (rc == SF_OK) rc = launch_batch(ds, p, 1, &c, nullptr, stream);
      }
      (void)hipEventRecord(e1, stream);
      if (hipEventSynchronize(e1) != hipSuccess) rc = fail(SF_EHIP, "hipEventSynchronize failed");
      float ms = 0.0f;
      if (rc == SF_OK && hipEventElapsedTime(&ms, e0, e1) == hipSuccess && ms / 2 < best_t) {
        best_t = ms / 2;
        best_c = c;
      }
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  *best = best_c;
  if (best_ms) *best_ms = best_t;
  return SF_OK;
}

}  // namespace sf
