// Standalone AES-128-CTR over an arbitrary device buffer (encrypt_private).
// Each lane produces one 16-byte keystream block E_K(ctr0 + first + i) from
// the LDS round tables and XORs it into 16 input bytes (coalesced 16-byte
// loads and stores); the trailing partial block is handled byte by byte.
#include "sf_internal.h"

namespace sf {
namespace {

constexpr int kThreads = 256;

struct CtrArgs {
  const uint8_t *in;
  uint8_t *out;
  uint64_t nbytes;
  uint64_t first;
  const uint32_t *aes_t0;
  AesArgs aes;
};

__global__ __launch_bounds__(kThreads) void ctr_kernel(CtrArgs a) {
  __shared__ AesLds s_aes;
  aes_load_tables(s_aes, a.aes_t0, a.aes.key, threadIdx.x, kThreads);
  __syncthreads();
  const uint64_t nblk = (a.nbytes + 15u) / 16u;
  for (uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x; i < nblk; i += (uint64_t)gridDim.x * kThreads) {
    uint32_t w0, w1, w2, w3;
    aes_counter(a.aes.ctr_hi, a.aes.ctr_lo, a.first + i, w0, w1, w2, w3);
    aes_encrypt(w0, w1, w2, w3, s_aes);
    const uint64_t off = 16u * i;
    if (off + 16u <= a.nbytes) {
      uint4 v = *reinterpret_cast<const uint4 *>(a.in + off);
      v.x ^= w0;
      v.y ^= w1;
      v.z ^= w2;
      v.w ^= w3;
      *reinterpret_cast<uint4 *>(a.out + off) = v;
    } else {
      const uint64_t lo = (uint64_t)w0 | ((uint64_t)w1 << 32), hi = (uint64_t)w2 | ((uint64_t)w3 << 32);
      for (uint64_t j = off; j < a.nbytes; ++j) {
        const uint32_t k = (uint32_t)(j - off);
        const uint8_t ks = (uint8_t)((k < 8u ? lo >> (8u * k) : hi >> (8u * (k - 8u))) & 0xffu);
        a.out[j] = (uint8_t)(a.in[j] ^ ks);
      }
    }
  }
}

}  // namespace

int launch_ctr(const DeviceState &ds, const AesArgs &aes, uint64_t first_block, const uint8_t *in, uint8_t *out,
               size_t nbytes, hipStream_t stream) {
  if (((uintptr_t)in | (uintptr_t)out) & 15u) return fail(SF_EINVAL, "buffers must be 16-byte aligned");
  CtrArgs a;
  a.in = in;
  a.out = out;
  a.nbytes = nbytes;
  a.first = first_block;
  a.aes_t0 = ds.d_aes_t0;
  a.aes = aes;
  const uint64_t nblk = (nbytes + 15u) / 16u;
  uint64_t grid = (nblk + kThreads - 1) / kThreads;
  const uint64_t cap = (uint64_t)ds.num_cu * 8u;
  if (grid > cap) grid = cap;
  hipLaunchKernelGGL(ctr_kernel, dim3((unsigned)grid), dim3(kThreads), 0, stream, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "ctr_kernel launch");
  return SF_OK;
}

}  // namespace sf
